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
// Tiles (variants, chosen per stage shape by the autotuner): 64 to 256
// right-hand sides x 64 or 128 complex output rows per workgroup of 4 or 8
// waves; the reduction is staged through LDS in chunks of 16 complex entries,
// optionally with one or two chunks of register prefetch or double-buffered
// LDS.  Global loads are branch-free (addresses clamped into the block, zero
// selected when the chunk is moved to LDS), so a chunk's loads are all in
// flight together and stay in flight during the matrix-core work.
// Arithmetic modes:
//   F32     v_mfma_f32_32x32x2_f32, one complex k per instruction; the chunk
//           sums are added to the running sums (two-level summation);
//   F32 3M  the same instruction on three real products (Gauss), 6 instead
//           of 8 real flops of matrix-core work per complex multiply-add;
//   BF16X3  v_mfma_f32_32x32x16_bf16, eight complex k per instruction; every
//           operand is split as hi + lo (both BF16) and the product is
//           hi*hi + hi*lo + lo*hi with FP32 accumulation.
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

constexpr int KCH = 16;      // reduction chunk (complex entries) of every variant
constexpr int PA = KCH + 4;  // LDS pitch (words) of the state operand rows

// LDS word of (output row mrow, real/imaginary output column d, 4-word group
// g of the chunk) in the block operand.  Each output row holds 2 x 16 words;
// the 16-byte groups are XOR-swizzled by the row so that the 16-byte reads of
// 32 consecutive real columns, and the 16-byte writes of consecutive rows,
// spread over the banks (conflict-free reads, at most 2-way writes).
__device__ __forceinline__ int bidx(int mrow, int d, int g) {
  return mrow * (2 * KCH) + d * KCH + (((g ^ mrow ^ (mrow >> 2)) & 3) << 2);
}

// Padded alternative for the FP32 kernels (whose LDS budget allows it): one
// row of PA words per real output column 2 mrow + d; 16-byte reads of
// consecutive rows are conflict-free and the offsets fold into immediates.
__device__ __forceinline__ int bidx_pad(int mrow, int d, int g) { return (2 * mrow + d) * PA + 4 * g; }

// Tile shape of a kernel variant: TNV right-hand sides x TMV complex output
// rows per workgroup of NTH threads; each wave owns RT x CT matrix-core tiles
// of 32 right-hand sides x 32 real columns.  PF prefetches the next chunk
// into registers during the matrix-core work; DB (which implies PF) also
// double-buffers the LDS so that one barrier per chunk separates the phases.
template <int TNV_, int TMV_, int NTH_, int RT_, int CT_, bool PF_, bool DB_, bool PF2_ = false>
struct Shape {
  static constexpr int TNV = TNV_, TMV = TMV_, NTH = NTH_, RT = RT_, CT = CT_;
  static constexpr bool PF = PF_ || DB_ || PF2_, DB = DB_;
  static constexpr bool PF2 = PF2_ && !DB_;  // two chunks of register prefetch (single LDS buffer)
  static constexpr int WR = TNV / (32 * RT);      // waves along right-hand sides
  static constexpr int WC = 2 * TMV / (32 * CT);  // waves along real columns
  static_assert(WR * WC * 64 == NTH, "the waves must cover the tile");
  static constexpr int EA = TNV * KCH / NTH;  // state entries per thread per chunk
  static constexpr int EB = TMV * 4 / NTH;    // (row, group) pairs of the block per thread per chunk
  static_assert(EA * NTH == TNV * KCH && EB * NTH == TMV * 4 && NTH % KCH == 0, "load mapping");
  static constexpr int NB = DB ? 2 : 1;  // LDS buffers
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
// Each chunk moves a TNV x 16 tile of the input state (A) and a 16 x TMV
// tile of the block (B) into registers, consecutive lanes on consecutive
// memory:
//   A:            k = tid % 16, n = tid / 16 + j (NTH / 16)
//   B forward:    pair p = tid + j NTH: row m = p % TMV, group g = p / TMV;
//                 the 4 entries W(m, 4g .. 4g+3) (lanes along m)
//   B adjoint:    pair p = tid + j NTH: group g = p % 4, row k' = p / 4;
//                 the 4 entries W(4g .. 4g+3, k') (contiguous)
template <class S, bool ADJ, typename WT>
struct Loader {
  float2 a[S::EA];
  WT b[S::EB][4];
  uint32_t ok;  // bit j: a[j] in range; bit EA + 4 j + i: b[j][i] in range
  static_assert(S::EA + 4 * S::EB <= 32, "predicate bits");
  // Branch-free: every lane loads from an address clamped into the block
  // (row, column and right-hand side indices clamped to their last valid
  // value); the entries outside are zeroed by finish(), on a copy made when
  // the chunk is moved to LDS.  A guarded load would sit in an exec-masked
  // branch, and a select right after it would consume it: either makes the
  // compiler wait for the load on the spot, so the prefetch of the next
  // chunk would not overlap the matrix-core work.  For the same reason the
  // kernels prefetch unconditionally: a chunk past the end reads clamped
  // (valid, recently read) addresses and comes out all zero.  Needs R >= 1,
  // Q >= 1 (the kernels skip the reduction otherwise) and nrhs >= 1 (checked
  // by the launcher).
  __device__ __forceinline__ void load(const BlockDesc& d, const float2* __restrict__ in, int64_t ld_in,
                                       const WT* __restrict__ Wb, int R, int Q, int r0, int n0, int q0,
                                       int nrhs) {
    constexpr int NTH = S::NTH, TMV = S::TMV;
    const int tid = threadIdx.x;
    ok = 0;
    {
      const int k = tid % KCH, n = tid / KCH;
      const int q = q0 + k;
      const int qc = min(q, Q - 1);
      const int32_t row = ADJ ? grp_row(d, qc) : d.in_row + qc;
#pragma unroll
      for (int j = 0; j < S::EA; ++j) {
        const int gn = n0 + n + j * (NTH / KCH);
        a[j] = in[(int64_t)min(gn, nrhs - 1) * ld_in + row];
        ok |= (uint32_t)(gn < nrhs && q < Q) << j;
      }
    }
#pragma unroll
    for (int j = 0; j < S::EB; ++j) {
      const int p = tid + j * NTH;
      if (!ADJ) {
        const int m = r0 + p % TMV, q = q0 + 4 * (p / TMV);
        const int mc = min(m, R - 1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          b[j][i] = Wb[(int64_t)min(q + i, Q - 1) * d.M + mc];
          ok |= (uint32_t)(m < R && q + i < Q) << (S::EA + 4 * j + i);
        }
      } else {
        const int mr = q0 + 4 * (p % 4), kout = r0 + p / 4;
        const int64_t base = (int64_t)min(kout, R - 1) * d.M;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          b[j][i] = Wb[base + min(mr + i, Q - 1)];
          ok |= (uint32_t)(kout < R && mr + i < Q) << (S::EA + 4 * j + i);
        }
      }
    }
  }
  // Zero the entries outside the block.
  __device__ __forceinline__ void finish() {
#pragma unroll
    for (int j = 0; j < S::EA; ++j)
      if (!((ok >> j) & 1)) a[j] = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < S::EB; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (!((ok >> (S::EA + 4 * j + i)) & 1)) b[j][i] = WT{};
  }
  // LDS row and group of pair j.
  __device__ __forceinline__ static void pair_pos(int j, int& mrow, int& g) {
    const int p = threadIdx.x + j * S::NTH;
    if (!ADJ) {
      mrow = p % S::TMV;
      g = p / S::TMV;
    } else {
      mrow = p / 4;
      g = p % 4;
    }
  }
};

// ------------------------------------------------------------------ FP32
// Wave w covers right-hand sides wn = (w % WR) * 32 RT and real columns
// wm = (w / WR) * 32 CT.  One MFMA consumes one complex k: lanes 0-31 the
// real parts (plane 0), lanes 32-63 the imaginary parts (plane 1).
template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_f32(const BlockDesc* __restrict__ blk,
                                                      const float2* __restrict__ W,
                                                      const float2* __restrict__ in, int64_t ld_in,
                                                      float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                      const float* __restrict__ scale, int mtiles, int ntiles,
                                                      int64_t total) {
  constexpr int NTH = S::NTH, TMV = S::TMV, TNV = S::TNV, RT = S::RT, CT = S::CT, NB = S::NB;
  __shared__ __attribute__((aligned(16))) float As[NB][2][TNV * PA];        // [buf][re|im][n][k]
  // block operand: [buf][plane][bidx_pad], two planes of 2 TMV x PA words
  constexpr int BPL = 2 * TMV * PA;
  __shared__ __attribute__((aligned(16))) float Bs[NB][2 * BPL];
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
  const float2* Wb = W + d.w_off;
  using LD = Loader<S, ADJ, float2>;
  LD ld;
  auto stash = [&](int buf) {
    LD c = ld;
    c.finish();
    const int k = tid % KCH, n = tid / KCH;
#pragma unroll
    for (int j = 0; j < S::EA; ++j) {
      As[buf][0][(n + j * (NTH / KCH)) * PA + k] = c.a[j].x;
      As[buf][1][(n + j * (NTH / KCH)) * PA + k] = c.a[j].y;
    }
#pragma unroll
    for (int j = 0; j < S::EB; ++j) {
      int mrow, g;
      LD::pair_pos(j, mrow, g);
      const float2* w = c.b[j];
      // forward B(2k+c, 2m+d): c=0: (Wr, Wi), c=1: (-Wi, Wr); the adjoint uses conj(W)
      const float s = ADJ ? -1.f : 1.f;
      *reinterpret_cast<float4*>(&Bs[buf][bidx_pad(mrow, 0, g)]) = make_float4(w[0].x, w[1].x, w[2].x, w[3].x);
      *reinterpret_cast<float4*>(&Bs[buf][bidx_pad(mrow, 1, g)]) =
          make_float4(s * w[0].y, s * w[1].y, s * w[2].y, s * w[3].y);
      *reinterpret_cast<float4*>(&Bs[buf][BPL + bidx_pad(mrow, 0, g)]) =
          make_float4(-s * w[0].y, -s * w[1].y, -s * w[2].y, -s * w[3].y);
      *reinterpret_cast<float4*>(&Bs[buf][BPL + bidx_pad(mrow, 1, g)]) = make_float4(w[0].x, w[1].x, w[2].x, w[3].x);
    }
  };
  // Two-level summation: the matrix cores sum one chunk into p, which is then
  // added to the running sums; the rounding error grows with the chunk
  // length plus the number of chunks instead of with the full reduction.
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  const int kk = lane >> 5, li = lane & 31;
  auto compute = [&](int buf) {
    v16f p[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) p[a][c] = v16f{};
#pragma unroll
    for (int kb = 0; kb < KCH; kb += 4) {
      float4 av[RT], bv[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a)
        av[a] = *reinterpret_cast<const float4*>(&As[buf][kk][(wn + 32 * a + li) * PA + kb]);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = wm + 32 * c + li;
        bv[c] = *reinterpret_cast<const float4*>(&Bs[buf][kk * BPL + bidx_pad(col >> 1, col & 1, kb >> 2)]);
      }
      // consecutive instructions go to different accumulator tiles
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].x, bv[c].x, p[a][c], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].y, bv[c].y, p[a][c], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].z, bv[c].z, p[a][c], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) p[a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a].w, bv[c].w, p[a][c], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[a][c] += p[a][c];
  };
  if (Q > 0) {  // (uniform) an empty reduction leaves the sums at zero
    if (S::DB) {
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      stash(0);
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, KCH, nrhs);
      __syncthreads();
      for (int q0 = 0, cur = 0; q0 < Q; q0 += KCH, cur ^= 1) {
        // Buffer cur^1 was last read before the previous barrier: refill it
        // (past the last chunk with zeros that are never read).
        stash(cur ^ 1);
        ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + 2 * KCH, nrhs);
        compute(cur);
        __syncthreads();
      }
    } else if (S::PF2) {
      LD ahead;  // chunk q0 + 2 KCH is loading while chunk q0 is summed
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      ahead.load(d, in, ld_in, Wb, R, Q, r0, n0, KCH, nrhs);
      for (int q0 = 0; q0 < Q; q0 += KCH) {
        stash(0);
        __syncthreads();
        ld = ahead;
        ahead.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + 2 * KCH, nrhs);
        compute(0);
        __syncthreads();
      }
    } else {
      if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      for (int q0 = 0; q0 < Q; q0 += KCH) {
        if (!S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
        stash(0);
        __syncthreads();
        if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KCH, nrhs);
        compute(0);
        __syncthreads();
      }
    }
  }
  store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// ------------------------------------------------------------------ FP32, 3 real products
// The complex product as three real products (Gauss): with X = Xr + i Xi
// and B = Br + i Bi,
//   T1 = Xr Br,  T2 = Xi Bi,  T3 = (Xr + Xi)(Br + Bi),
//   Re = T1 - T2,  Im = T3 - T1 - T2,
// i.e. 6 real flops of matrix-core work per complex multiply-add instead of
// the 8 of the real embedding.  Each MFMA consumes two complex k (lanes 0-31
// k, lanes 32-63 k + 4 of a group of 8).  The wave tile is 32 RT right-hand
// sides x 32 CT complex output rows; T1..T3 are summed in two levels like the
// other FP32 kernels.
template <int TNV_, int TMV_, int NTH_, int RT_, int CT_, bool PF_, bool DB_>
struct Shape3 {
  static constexpr int TNV = TNV_, TMV = TMV_, NTH = NTH_, RT = RT_, CT = CT_;
  static constexpr bool PF = PF_ || DB_, DB = DB_;
  static constexpr int WR = TNV / (32 * RT);  // waves along right-hand sides
  static constexpr int WC = TMV / (32 * CT);  // waves along complex output rows
  static_assert(WR * WC * 64 == NTH, "the waves must cover the tile");
  static constexpr int EA = TNV * KCH / NTH;
  static constexpr int EB = TMV * 4 / NTH;
  static_assert(EA * NTH == TNV * KCH && EB * NTH == TMV * 4 && NTH % KCH == 0, "load mapping");
  static constexpr int NB = DB ? 2 : 1;
};

template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_f32_3m(const BlockDesc* __restrict__ blk,
                                                         const float2* __restrict__ W,
                                                         const float2* __restrict__ in, int64_t ld_in,
                                                         float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                         const float* __restrict__ scale, int mtiles, int ntiles,
                                                         int64_t total) {
  constexpr int NTH = S::NTH, TMV = S::TMV, TNV = S::TNV, RT = S::RT, CT = S::CT, NB = S::NB;
  __shared__ __attribute__((aligned(16))) float As[NB][3][TNV * PA];  // [buf][Xr|Xi|Xr+Xi][n][k]
  __shared__ __attribute__((aligned(16))) float Bs[NB][3][TMV * PA];  // [buf][Br|Bi|Br+Bi][m][k]
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
  const float2* Wb = W + d.w_off;
  using LD = Loader<S, ADJ, float2>;
  LD ld;
  auto stash = [&](int buf) {
    LD c = ld;
    c.finish();
    const int k = tid % KCH, n = tid / KCH;
#pragma unroll
    for (int j = 0; j < S::EA; ++j) {
      const int e = (n + j * (NTH / KCH)) * PA + k;
      const float2 v = c.a[j];
      As[buf][0][e] = v.x;
      As[buf][1][e] = v.y;
      As[buf][2][e] = v.x + v.y;
    }
#pragma unroll
    for (int j = 0; j < S::EB; ++j) {
      int mrow, g;
      LD::pair_pos(j, mrow, g);
      const float2* w = c.b[j];
      const float s = ADJ ? -1.f : 1.f;  // B = W (forward) or conj(W) (adjoint)
      const int e = mrow * PA + 4 * g;
      *reinterpret_cast<float4*>(&Bs[buf][0][e]) = make_float4(w[0].x, w[1].x, w[2].x, w[3].x);
      *reinterpret_cast<float4*>(&Bs[buf][1][e]) = make_float4(s * w[0].y, s * w[1].y, s * w[2].y, s * w[3].y);
      *reinterpret_cast<float4*>(&Bs[buf][2][e]) =
          make_float4(w[0].x + s * w[0].y, w[1].x + s * w[1].y, w[2].x + s * w[2].y, w[3].x + s * w[3].y);
    }
  };
  v16f acc[3][RT][CT];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[t][a][c] = v16f{};
  const int kk = lane >> 5, li = lane & 31;
  auto compute = [&](int buf) {
    v16f p[3][RT][CT];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) p[t][a][c] = v16f{};
#pragma unroll
    for (int kb = 0; kb < KCH; kb += 8) {
      const int ko = kb + 4 * kk;
      float4 av[3][RT], bv[3][CT];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
#pragma unroll
        for (int a = 0; a < RT; ++a)
          av[t][a] = *reinterpret_cast<const float4*>(&As[buf][t][(wn + 32 * a + li) * PA + ko]);
#pragma unroll
        for (int c = 0; c < CT; ++c)
          bv[t][c] = *reinterpret_cast<const float4*>(&Bs[buf][t][(wm + 32 * c + li) * PA + ko]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
          for (int a = 0; a < RT; ++a)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
              const float x = j == 0 ? av[t][a].x : j == 1 ? av[t][a].y : j == 2 ? av[t][a].z : av[t][a].w;
              const float y = j == 0 ? bv[t][c].x : j == 1 ? bv[t][c].y : j == 2 ? bv[t][c].z : bv[t][c].w;
              p[t][a][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, p[t][a][c], 0, 0, 0);
            }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][a][c] += p[t][a][c];
  };
  if (Q > 0) {  // (uniform) an empty reduction leaves the sums at zero
    if (S::DB) {
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      stash(0);
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, KCH, nrhs);
      __syncthreads();
      for (int q0 = 0, cur = 0; q0 < Q; q0 += KCH, cur ^= 1) {
        // Buffer cur^1 was last read before the previous barrier: refill it
        // (past the last chunk with zeros that are never read).
        stash(cur ^ 1);
        ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + 2 * KCH, nrhs);
        compute(cur);
        __syncthreads();
      }
    } else {
      if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      for (int q0 = 0; q0 < Q; q0 += KCH) {
        if (!S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
        stash(0);
        __syncthreads();
        if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KCH, nrhs);
        compute(0);
        __syncthreads();
      }
    }
  }
  // Re = T1 - T2, Im = T3 - T1 - T2; lane li holds complex row wm + 32 c + li
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int m = r0 + wm + 32 * c + li;
    if (m >= R) continue;
    const int32_t row = ADJ ? d.in_row + m : grp_row(d, m);
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = n0 + wn + 32 * a + 8 * (j >> 2) + 4 * kk + (j & 3);
        if (n < nrhs) {
          const float t1 = acc[0][a][c][j], t2 = acc[1][a][c][j], t3 = acc[2][a][c][j];
          out[(int64_t)n * ld_out + row] = make_float2((t1 - t2) * sc, (t3 - t1 - t2) * sc);
        }
      }
  }
}

// ------------------------------------------------------------------ BF16 x3
// LDS words hold two BF16 values along the reduction: the state word (n, k)
// is (Re, Im) of x(n, k); the block words are the matching pairs of the
// embedding.  The split products carry ~2^-16 relative error, so the partial
// sums go straight into the matrix-core accumulators (no compensation).
template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_bf16x3(const BlockDesc* __restrict__ blk,
                                                         const uint2* __restrict__ W,  // (re_hi,im_hi | re_lo,im_lo)
                                                         const float2* __restrict__ in, int64_t ld_in,
                                                         float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                         const float* __restrict__ scale, int mtiles, int ntiles,
                                                         int64_t total) {
  constexpr int NTH = S::NTH, TMV = S::TMV, TNV = S::TNV, RT = S::RT, CT = S::CT, NB = S::NB;
  __shared__ __attribute__((aligned(16))) uint32_t Ah[NB][TNV * PA], Al[NB][TNV * PA];
  __shared__ __attribute__((aligned(16))) uint32_t Bh[NB][TMV * 2 * KCH], Bl[NB][TMV * 2 * KCH];
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
  using LD = Loader<S, ADJ, uint2>;
  LD ld;
  auto stash = [&](int buf) {  // registers -> LDS (state split into BF16 hi/lo here)
    LD c = ld;
    c.finish();
    const int k = tid % KCH, n = tid / KCH;
#pragma unroll
    for (int j = 0; j < S::EA; ++j) {
      uint32_t rh, rl, ih, il;
      split_bf(c.a[j].x, rh, rl);
      split_bf(c.a[j].y, ih, il);
      Ah[buf][(n + j * (NTH / KCH)) * PA + k] = rh | (ih << 16);
      Al[buf][(n + j * (NTH / KCH)) * PA + k] = rl | (il << 16);
    }
#pragma unroll
    for (int j = 0; j < S::EB; ++j) {
      int mrow, g;
      LD::pair_pos(j, mrow, g);
      uint32_t h0[4], h1[4], l0[4], l1[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint2 w = c.b[j][i];
        const uint32_t reh = w.x & 0xffffu, imh = w.x >> 16, rel = w.y & 0xffffu, iml = w.y >> 16;
        if (!ADJ) {  // column 2m: (Wr, -Wi);  column 2m+1: (Wi, Wr)
          h0[i] = reh | ((imh ^ 0x8000u) << 16);
          h1[i] = imh | (reh << 16);
          l0[i] = rel | ((iml ^ 0x8000u) << 16);
          l1[i] = iml | (rel << 16);
        } else {  // conj(W): column 2k': (Wr, Wi);  column 2k'+1: (-Wi, Wr)
          h0[i] = reh | (imh << 16);
          h1[i] = (imh ^ 0x8000u) | (reh << 16);
          l0[i] = rel | (iml << 16);
          l1[i] = (iml ^ 0x8000u) | (rel << 16);
        }
      }
      *reinterpret_cast<uint4*>(&Bh[buf][bidx(mrow, 0, g)]) = make_uint4(h0[0], h0[1], h0[2], h0[3]);
      *reinterpret_cast<uint4*>(&Bh[buf][bidx(mrow, 1, g)]) = make_uint4(h1[0], h1[1], h1[2], h1[3]);
      *reinterpret_cast<uint4*>(&Bl[buf][bidx(mrow, 0, g)]) = make_uint4(l0[0], l0[1], l0[2], l0[3]);
      *reinterpret_cast<uint4*>(&Bl[buf][bidx(mrow, 1, g)]) = make_uint4(l1[0], l1[1], l1[2], l1[3]);
    }
  };
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  const int kh = lane >> 5, li = lane & 31;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kb = 0; kb < KCH; kb += 8) {
      // lane holds real-k 8*kh .. 8*kh+7 of this step = complex k kb + 4*kh .. +3
      const int ko = kb + 4 * kh;
      bf16x8 ah[RT], al[RT], bh[CT], bl[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        const int e = (wn + 32 * a + li) * PA + ko;
        ah[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Ah[buf][e]));
        al[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Al[buf][e]));
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int col = wm + 32 * c + li;
        const int e = bidx(col >> 1, col & 1, ko >> 2);
        bh[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bh[buf][e]));
        bl[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bl[buf][e]));
      }
      // consecutive instructions go to different accumulator tiles
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[c], acc[a][c], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[c], acc[a][c], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[c], acc[a][c], 0, 0, 0);
    }
  };
  if (Q > 0) {  // (uniform) an empty reduction leaves the sums at zero
    if (S::DB) {
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      stash(0);
      ld.load(d, in, ld_in, Wb, R, Q, r0, n0, KCH, nrhs);
      __syncthreads();
      for (int q0 = 0, cur = 0; q0 < Q; q0 += KCH, cur ^= 1) {
        // Buffer cur^1 was last read before the previous barrier: refill it
        // (past the last chunk with zeros that are never read).
        stash(cur ^ 1);
        ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + 2 * KCH, nrhs);
        compute(cur);
        __syncthreads();
      }
    } else {
      if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, 0, nrhs);
      for (int q0 = 0; q0 < Q; q0 += KCH) {
        if (!S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0, nrhs);
        stash(0);
        __syncthreads();
        if (S::PF) ld.load(d, in, ld_in, Wb, R, Q, r0, n0, q0 + KCH, nrhs);
        compute(0);
        __syncthreads();
      }
    }
  }
  store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// Kernel variants: Shape<TNV, TMV, NTH, RT, CT, PF, DB>.
using F0 = Shape<64, 64, 256, 1, 2, false, false>;
using F1 = Shape<64, 64, 256, 1, 2, true, false>;
using F2 = Shape<128, 64, 256, 2, 2, true, false>;
using F3 = Shape<64, 64, 256, 1, 2, true, true>;
using F4 = Shape<128, 64, 256, 2, 2, true, true>;
using F5 = Shape<128, 128, 512, 2, 2, true, true>;
// FP32 with three real products (k_stage_f32_3m)
using G6 = Shape3<64, 64, 256, 1, 1, false, false>;
using G7 = Shape3<64, 64, 256, 1, 1, true, false>;
using G8 = Shape3<64, 64, 256, 1, 1, true, true>;
// FP32 with two chunks of register prefetch
using F9 = Shape<64, 64, 256, 1, 2, true, false, true>;
using F10 = Shape<128, 64, 256, 2, 2, true, false, true>;
using B0 = Shape<64, 64, 256, 1, 2, false, false>;
using B1 = Shape<128, 64, 256, 2, 2, true, false>;
using B2 = Shape<256, 128, 512, 2, 4, true, false>;
using B3 = Shape<128, 128, 256, 2, 4, true, false>;
using B4 = Shape<128, 64, 256, 2, 2, true, true>;
using B5 = Shape<256, 128, 512, 2, 4, true, true>;
using B6 = Shape<128, 128, 256, 2, 4, true, true>;

struct VariantDims {
  int tnv, tmv, nth;
};
template <class S>
constexpr VariantDims dims_of() {
  return {S::TNV, S::TMV, S::NTH};
}

VariantDims variant_dims(int prec, int v) {
  if (prec == MBF_C64) {
    switch (v) {
      case 0: return dims_of<F0>();
      case 1: return dims_of<F1>();
      case 2: return dims_of<F2>();
      case 3: return dims_of<F3>();
      case 4: return dims_of<F4>();
      case 5: return dims_of<F5>();
      case 6: return dims_of<G6>();
      case 7: return dims_of<G7>();
      case 8: return dims_of<G8>();
      case 9: return dims_of<F9>();
      default: return dims_of<F10>();
    }
  }
  switch (v) {
    case 0: return dims_of<B0>();
    case 1: return dims_of<B1>();
    case 2: return dims_of<B2>();
    case 3: return dims_of<B3>();
    case 4: return dims_of<B4>();
    case 5: return dims_of<B5>();
    default: return dims_of<B6>();
  }
}

}  // namespace

bool use_mfma(const DevPart&, int, int64_t nrhs, int prec) {
  if (prec == MBF_C64_SPLIT_BF16) return true;
  if (prec == MBF_C64) return nrhs > 32;  // up to 32 RHS: the 16 x 16 kernel (stage_r16.hip)
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
  // Untuned defaults: the small FP32 tile; for BF16 x3 the double-buffered
  // 256 x 128 tile when the right-hand sides fill it, the 128 x 64 one for
  // mid-size batches, the 64 x 64 one for small batches.
  if (prec == MBF_C64) return 0;
  return nrhs >= 192 ? 5 : nrhs > 64 ? 4 : 0;
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
      case 0: MBF_LAUNCH(k_stage_f32, float2, F0); break;
      case 1: MBF_LAUNCH(k_stage_f32, float2, F1); break;
      case 2: MBF_LAUNCH(k_stage_f32, float2, F2); break;
      case 3: MBF_LAUNCH(k_stage_f32, float2, F3); break;
      case 4: MBF_LAUNCH(k_stage_f32, float2, F4); break;
      case 5: MBF_LAUNCH(k_stage_f32, float2, F5); break;
      case 6: MBF_LAUNCH(k_stage_f32_3m, float2, G6); break;
      case 7: MBF_LAUNCH(k_stage_f32_3m, float2, G7); break;
      case 8: MBF_LAUNCH(k_stage_f32_3m, float2, G8); break;
      case 9: MBF_LAUNCH(k_stage_f32, float2, F9); break;
      default: MBF_LAUNCH(k_stage_f32, float2, F10); break;
    }
  } else {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_bf16x3, uint2, B0); break;
      case 1: MBF_LAUNCH(k_stage_bf16x3, uint2, B1); break;
      case 2: MBF_LAUNCH(k_stage_bf16x3, uint2, B2); break;
      case 3: MBF_LAUNCH(k_stage_bf16x3, uint2, B3); break;
      case 4: MBF_LAUNCH(k_stage_bf16x3, uint2, B4); break;
      case 5: MBF_LAUNCH(k_stage_bf16x3, uint2, B5); break;
      default: MBF_LAUNCH(k_stage_bf16x3, uint2, B6); break;
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
  if (nrhs < 1) return {MBF_ERR_INVALID_ARG, "MFMA stage: nrhs < 1"};
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
