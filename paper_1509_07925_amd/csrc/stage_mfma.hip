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

// Split state of the BF16 x3 kernels: each complex entry x becomes the two
// words hi = Re_hi | Im_hi << 16 and lo = Re_lo | Im_lo << 16 (BF16 bits),
// stored where the FP32 (Re, Im) pair would be: the 8 bytes of entry (n, row)
// are (hi, lo).  kInSplit / kOutSplit: the input / output state of a launch
// is split.
constexpr int kInSplit = 1, kOutSplit = 2;

// store_out writing the split state.  Lane pairs (2i, 2i+1) hold the real
// and imaginary part of one complex entry; each lane splits its value, the
// pair swaps one half (DPP quad permutation 1,0,3,2), and the even lane
// stores the hi word, the odd lane the lo word: the addresses, hence the
// coalescing, of the FP32 store.
template <bool ADJ, int RT, int CT>
__device__ __forceinline__ void store_out_split(const BlockDesc& d, int R, int r0, int n0,
                                                const v16f (&acc)[RT][CT], int wn, int wm, float2* __restrict__ out,
                                                int64_t ld_out, int nrhs, const float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const bool odd = lane & 1;
  uint32_t* o = reinterpret_cast<uint32_t*>(out);
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int col = wm + c * 32 + (lane & 31);
    const int m = r0 + (col >> 1);
    const bool mok = m < R;  // uniform over each lane pair
    const int32_t row = ADJ ? d.in_row + min(m, R - 1) : grp_row(d, min(m, R - 1));
    const float sc = scale ? scale[row] : 1.0f;
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int n = n0 + wn + 32 * a + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        uint32_t hi, lo;
        // The product is rounded first, as the FP32 store rounds it: the empty
        // asm keeps the compiler from fusing it into the lo residual (the
        // split is then that of the FP32 value, bit for bit).
        float x = acc[a][c][j] * sc;
        asm volatile("" : "+v"(x));
        split_bf(x, hi, lo);
        const uint32_t recv = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(odd ? hi : lo), 0xB1, 0xF, 0xF, false);
        const uint32_t w = odd ? (recv | (lo << 16)) : (hi | (recv << 16));
        if (mok && n < nrhs) o[2 * ((int64_t)n * ld_out + row) + (col & 1)] = w;
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
template <class S, bool ADJ, typename WT, bool LOAD_A = true>
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
    if constexpr (LOAD_A) {
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
    if constexpr (LOAD_A) {
#pragma unroll
      for (int j = 0; j < S::EA; ++j)
        if (!((ok >> j) & 1)) a[j] = make_float2(0.f, 0.f);
    }
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
                                                      int64_t total, int /*flags*/) {
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
                                                         int64_t total, int /*flags*/) {
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
// Block operand of a chunk (registers -> LDS): the BF16 pairs of the real
// embedding, hi and lo parts in separate arrays (bidx layout).
template <bool ADJ, class S, class LD>
__device__ __forceinline__ void stash_block_bf16(const LD& c, uint32_t* __restrict__ Bh, uint32_t* __restrict__ Bl) {
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
    *reinterpret_cast<uint4*>(&Bh[bidx(mrow, 0, g)]) = make_uint4(h0[0], h0[1], h0[2], h0[3]);
    *reinterpret_cast<uint4*>(&Bh[bidx(mrow, 1, g)]) = make_uint4(h1[0], h1[1], h1[2], h1[3]);
    *reinterpret_cast<uint4*>(&Bl[bidx(mrow, 0, g)]) = make_uint4(l0[0], l0[1], l0[2], l0[3]);
    *reinterpret_cast<uint4*>(&Bl[bidx(mrow, 1, g)]) = make_uint4(l1[0], l1[1], l1[2], l1[3]);
  }
}

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
                                                         int64_t total, int flags) {
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
    stash_block_bf16<ADJ, S>(c, Bh[buf], Bl[buf]);
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
  if (flags & kOutSplit)
    store_out_split<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
  else
    store_out<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
}

// ------------------------------------------------------------------ BF16 x3, split input
// Interior stages read a split state (kInSplit).  Both operands then move
// from memory into LDS by buffer loads that write LDS directly: no registers
// and no VALU work per chunk (per-lane offsets are fixed per tile, the chunk
// advances through the scalar offset), three chunks deep (chunks q + 1 and
// q + 2 load while q is summed).  The state operand is 2 right-hand sides x
// 16 reduction entries x (hi, lo) per load (two 128-byte runs), in LDS
// [n][8 groups of (hi, lo, hi, lo)] with the group of entries (2 g, 2 g + 1)
// at position g ^ ((n / 2) % 8), so that the 16-byte reads of 16 consecutive
// rows fall on distinct banks.  The block operand is read raw (see the block
// loads below); the real embedding (per output-column parity, a swap of the
// BF16 halves and a sign) is applied as
// the operands are read.  Every load reads whole 128-byte lines: the memory
// pipeline holds a bounded number of requests per CU, and loads that gather
// short pieces from many lines run several times slower.
// Reads past the block take clamped addresses, except the block operand's
// reduction entries past the end, which read zero (offsets past the buffer
// range); right-hand sides and output rows past the block are not stored.  Vector
// memory operations complete in issue order, so waiting until at most one
// chunk's loads are outstanding completes the chunk before it.  Loads are
// also issued past the last chunk (clamped, into buffers not read again) so
// that this count holds on every iteration.
template <class S>
struct DmaShape {
  static constexpr int NW = S::NTH / 64;            // waves
  static constexpr int NIA = S::TNV * 32 / S::NTH;  // state loads per wave per chunk
  static constexpr int NIB = S::TMV * 32 / S::NTH;  // block loads per wave per chunk (both planes)
  static constexpr int NI = NIA + NIB;
  static_assert(NIA * NW == S::TNV / 2 && NIB * NW == S::TMV / 2, "LDS load mapping");
  static_assert(NIA % 8 == 0 && NI <= 63 && S::TMV % 32 == 0, "LDS load mapping");
};

typedef int v4i __attribute__((ext_vector_type(4)));

// Raw buffer resource (stride 0) over [base, base + bytes): loads at offsets
// past the end return zero.
// (base and bytes are uniform; read from the first lane so that the compiler
// holds them in scalar registers, as the instruction requires)
__device__ __forceinline__ v4i buffer_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = reinterpret_cast<uint64_t>(base);
  return v4i{__builtin_amdgcn_readfirstlane((int)(uint32_t)b),
             __builtin_amdgcn_readfirstlane((int)((uint32_t)(b >> 32) & 0xffffu)),
             __builtin_amdgcn_readfirstlane((int)bytes), 0x00020000};
}

// One dword per lane from rs + voff + soff into LDS at lds + 4 lane (the
// buffer load's LDS form).  Written as assembly so that the compiler, which
// would otherwise make every later LDS read wait for all such loads, leaves
// the waits to the kernel (explicit s_waitcnt before the barriers that
// publish a buffer).  The instruction has no register result.
// The LDS address of a flat pointer into LDS is its low 32 bits (the LDS
// aperture's base is 4 GiB aligned).
__device__ __forceinline__ void lds_load_dword(v4i rs, const uint32_t* lds, uint32_t voff, uint32_t soff) {
  const uint32_t a = __builtin_amdgcn_readfirstlane((uint32_t)reinterpret_cast<uintptr_t>(lds));
  asm volatile("" : "+s"(soff));  // a register even when the offset is a known constant
  asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, %3 offen lds" ::"s"(a), "v"(voff), "s"(rs), "s"(soff)
               : "memory");
}

// s_waitcnt immediate: at most n vector-memory operations outstanding, no
// LDS operation outstanding (no wait on export counts).
constexpr int vm_lgkm0(int n) { return (n & 15) | (0x7 << 4) | ((n >> 4) << 14); }

template <bool ADJ, class S>
__global__ __launch_bounds__(S::NTH) void k_stage_bf16x3_dma(const BlockDesc* __restrict__ blk,
                                                             const uint2* __restrict__ W,
                                                             const float2* __restrict__ in, int64_t ld_in,
                                                             float2* __restrict__ out, int64_t ld_out, int nrhs,
                                                             const float* __restrict__ scale, int mtiles,
                                                             int ntiles, int64_t total, int flags) {
  constexpr int TMV = S::TMV, TNV = S::TNV, RT = S::RT, CT = S::CT;
  using DS = DmaShape<S>;
  // One array per buffer, each accessed through a constant address: the
  // compiler then knows which buffer a pending LDS load writes and does not
  // make reads of the other buffers wait for it.
  __shared__ __attribute__((aligned(16))) uint32_t As0[2][TNV * KCH], As1[2][TNV * KCH], As2[2][TNV * KCH];
  __shared__ __attribute__((aligned(16))) uint32_t Bs0[2][TMV * KCH], Bs1[2][TMV * KCH], Bs2[2][TMV * KCH];
  static_assert(2 * TMV * KCH == 64 * DmaShape<S>::NIB * (S::NTH / 64), "block loads fill the buffer");
  const Tile tl = map_tile(total, mtiles, ntiles);
  if (tl.b < 0) return;
  const BlockDesc d = blk[tl.b];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int r0 = tl.mt * TMV;
  if (r0 >= R) return;
  const int n0 = tl.nt * TNV;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wn = (wave % S::WR) * 32 * RT, wm = (wave / S::WR) * 32 * CT;
  // State loads: load t = wave NIA + i holds right-hand sides 2 t + l / 32;
  // lane l fills word p = l % 32 of its LDS row: group p / 4 holds entries
  // (2 g, 2 g + 1) with g = (p / 4) ^ (t % 8) (t % 8 = i % 8: NIA is a
  // multiple of 8), word p % 4 is (hi, lo, hi, lo)[...] of them.
  const int nl = lane >> 5, p32 = lane & 31;
  // reduction entry of lane l in loads with i % 8 = j
  auto ka = [&](int j) __attribute__((always_inline)) { return 2 * ((p32 >> 2) ^ j) + ((p32 >> 1) & 1); };
  const uint32_t pla = 4u * (lane & 1);  // hi / lo word
  // one buffer resource per wave, based at its first right-hand side
  // (offsets stay below 8 ld_in (2 NIA + 2) bytes: ld_in < 2^23)
  const bool full = n0 + TNV <= nrhs;  // (uniform) no right-hand side of the tile is clamped
  const int nb0 = min(n0 + 2 * wave * DS::NIA, nrhs - 1);
  const v4i rsa = buffer_rsrc(in + (int64_t)nb0 * ld_in, 0xffffffffu);
  const uint32_t stepa = 16u * (uint32_t)ld_in;  // bytes between consecutive loads' right-hand sides
  uint32_t va[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) va[j] = 8u * (uint32_t)(nl * ld_in + ka(j)) + pla;
  // block (W column-major M x K, 8 bytes per entry): output row (forward m,
  // adjoint k') clamped into the block, reduction word through the scalar offset
  const int M = d.M;
  // (range: the block, so that the past-the-end offset below reads zero)
  const v4i rsb = buffer_rsrc(W + d.w_off, 8u * (uint32_t)M * (uint32_t)d.K);
  // Block loads: each reads contiguous runs of the column-major block (hi and
  // lo words of consecutive entries, lanes alternating between them).
  //   forward: load t = wave NIB + i holds reduction entry k = t / (TMV / 32)
  //            and output rows m = 32 (t % (TMV / 32)) + l / 2 (256 bytes);
  //            LDS [k][m][hi, lo] (words 2 TMV k + 2 m + plane).
  //   adjoint: load t holds output columns k' = 2 t + l / 64 .. and reduction
  //            entries m = 2 g + w / 2 (two runs of 128 bytes); LDS
  //            [k'][8 groups of (hi, lo, hi, lo)], the group of m / 2 at
  //            position (m / 2) ^ ((k' / 2) % 8) so that 16-byte reads of 16
  //            consecutive columns fall on distinct banks.
  // forward: the entry k of a load is uniform (scalar offset); the lane part
  // repeats with period TMV / 32 in i (NIB is a multiple of it)
  constexpr int NVB = ADJ ? DS::NIB : (DS::NIB < TMV / 32 ? DS::NIB : TMV / 32);
  static_assert(ADJ || DS::NIB % NVB == 0, "block load pattern");
  uint32_t vb[NVB];
#pragma unroll
  for (int i = 0; i < NVB; ++i) {
    const int t = wave * DS::NIB + i;
    if (!ADJ) {
      const int m = 32 * (t % (TMV / 32)) + (lane >> 1);
      vb[i] = 8u * (uint32_t)min(r0 + m, R - 1) + 4u * (lane & 1);
    } else {
      const int r = 2 * t + (lane >> 5), p = lane & 31, g = (p >> 2) ^ (t & 7), w4 = p & 3;
      vb[i] = 8u * (uint32_t)(min(r0 + r, R - 1) * M + 2 * g + (w4 >> 1)) + 4u * (w4 & 1);
    }
  }
  auto kfw = [&](int i) __attribute__((always_inline)) { return (wave * DS::NIB + i) / (TMV / 32); };
  // Loads of a chunk: NI per wave, load j < NIA of the state, the rest of the
  // block.  The plan (uniform) holds what is common to a chunk's loads; the
  // input rows of [q0, q0 + 16) are contiguous from rowbase + q0 when the
  // chunk lies inside the block and inside one input group.
  struct Plan {
    int q0;
    int32_t rowbase;
    bool fasta, fast;
  };
  auto plan = [&](int q0) __attribute__((always_inline)) {
    Plan p{q0, d.in_row, false, q0 + KCH <= Q};
    p.fasta = full && p.fast;
    if (ADJ) {  // the group holding q0 (selects, as in grp_row)
      int32_t end = d.ms[1];
      p.rowbase = d.orow[0] - d.ms[0];
      if (q0 >= d.ms[1]) p.rowbase = d.orow[1] - d.ms[1], end = d.ms[2];
      if (q0 >= d.ms[2]) p.rowbase = d.orow[2] - d.ms[2], end = d.ms[3];
      if (q0 >= d.ms[3]) p.rowbase = d.orow[3] - d.ms[3], end = Q;
      p.fasta = p.fasta && q0 + KCH <= end;
    }
    return p;
  };
  auto dma = [&](uint32_t (*As)[TNV * KCH], uint32_t (*Bs)[TMV * KCH], const Plan& p, int j)
                 __attribute__((always_inline)) {
    const int q0 = p.q0;
    if (j < DS::NIA) {
      const int i = j;
      uint32_t* dst = &As[0][64 * (DS::NIA * wave + i)];
      if (p.fasta) {  // (uniform)
        lds_load_dword(rsa, dst, va[i & 7], 8u * (uint32_t)(p.rowbase + q0) + i * stepa);
      } else {
        const int q = min(q0 + ka(i & 7), Q - 1);
        const int32_t row = ADJ ? grp_row(d, q) : d.in_row + q;
        const int nr = min(n0 + 2 * (wave * DS::NIA + i) + nl, nrhs - 1) - nb0;
        lds_load_dword(rsa, dst, 8u * (uint32_t)(nr * ld_in + row) + pla, 0u);
      }
    } else {
      const int i = j - DS::NIA;
      uint32_t* dst = &Bs[0][64 * (DS::NIB * wave + i)];
      if (p.fast) {  // (uniform)
        if (ADJ)
          lds_load_dword(rsb, dst, vb[i % NVB], 8u * (uint32_t)q0);
        else
          lds_load_dword(rsb, dst, vb[i % NVB], 8u * (uint32_t)((q0 + kfw(i)) * M));
      } else {  // reduction entries past the block read zero (offset past the range)
        const int t = wave * DS::NIB + i;
        int q;
        if (!ADJ) {
          q = q0 + t / (TMV / 32);
        } else {
          const int pp = lane & 31, g = (pp >> 2) ^ (t & 7);
          q = q0 + 2 * g + ((pp & 3) >> 1);
        }
        const uint32_t off = ADJ ? vb[i % NVB] + 8u * (uint32_t)q0 : vb[i % NVB] + 8u * (uint32_t)(q * M);
        lds_load_dword(rsb, dst, q < Q ? off : 0xfffffff0u, 0u);
      }
    }
  };
  auto issue = [&](uint32_t (*As)[TNV * KCH], uint32_t (*Bs)[TMV * KCH], int q0) __attribute__((always_inline)) {
    const Plan p = plan(q0);
#pragma unroll
    for (int j = 0; j < DS::NI; ++j) dma(As, Bs, p, j);
  };
  v16f acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[a][c] = v16f{};
  const int kh = lane >> 5, li = lane & 31;
  // Embedding of a raw block word (Re | Im << 16) for this lane's real output
  // column 2 m + (li & 1): forward (Wr, -Wi) | (Wi, Wr), adjoint (conj W)
  // (Wr, Wi) | (-Wi, Wr); i.e. rotate by 16 bits for odd columns, then flip
  // one sign bit.
  const uint32_t rot = (li & 1) ? 16u : 0u;
  const uint32_t sgn = ADJ ? ((li & 1) ? 0x8000u : 0u) : ((li & 1) ? 0u : 0x80000000u);
  auto embed = [&](uint4 w) __attribute__((always_inline)) {
    uint32_t e[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) e[j] = __builtin_amdgcn_alignbit(e[j], e[j], rot) ^ sgn;
    return __builtin_bit_cast(bf16x8, make_uint4(e[0], e[1], e[2], e[3]));
  };
  auto compute = [&](const uint32_t (*As)[TNV * KCH], const uint32_t (*Bs)[TMV * KCH]) __attribute__((always_inline)) {
#pragma unroll
    for (int kb = 0; kb < KCH; kb += 8) {
      const int ko = kb + 4 * kh;
      bf16x8 ah[RT], al[RT], bh[CT], bl[CT];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        const int n = wn + 32 * a + li, sw = (n >> 1) & 7;
        const uint32_t* b = &As[0][0] + 32 * n;
        const uint4 u = *reinterpret_cast<const uint4*>(b + 4 * ((ko >> 1) ^ sw));
        const uint4 v = *reinterpret_cast<const uint4*>(b + 4 * (((ko >> 1) + 1) ^ sw));
        ah[a] = __builtin_bit_cast(bf16x8, make_uint4(u.x, u.z, v.x, v.z));
        al[a] = __builtin_bit_cast(bf16x8, make_uint4(u.y, u.w, v.y, v.w));
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int r = (wm + 32 * c + li) >> 1;  // output row (forward m, adjoint k') of the tile
        uint2 x0, x1, x2, x3;                   // (hi, lo) of reduction entries ko .. ko + 3
        if (!ADJ) {
          const uint32_t* b = &Bs[0][0] + 2 * TMV * ko + 2 * r;
          x0 = *reinterpret_cast<const uint2*>(b);
          x1 = *reinterpret_cast<const uint2*>(b + 2 * TMV);
          x2 = *reinterpret_cast<const uint2*>(b + 4 * TMV);
          x3 = *reinterpret_cast<const uint2*>(b + 6 * TMV);
        } else {
          const uint32_t* b = &Bs[0][0] + 32 * r;
          const int sw = (r >> 1) & 7;
          const uint4 u = *reinterpret_cast<const uint4*>(b + 4 * ((ko >> 1) ^ sw));
          const uint4 v = *reinterpret_cast<const uint4*>(b + 4 * (((ko >> 1) + 1) ^ sw));
          x0 = make_uint2(u.x, u.y);
          x1 = make_uint2(u.z, u.w);
          x2 = make_uint2(v.x, v.y);
          x3 = make_uint2(v.z, v.w);
        }
        bh[c] = embed(make_uint4(x0.x, x1.x, x2.x, x3.x));
        bl[c] = embed(make_uint4(x0.y, x1.y, x2.y, x3.y));
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
    const int nch = (Q + KCH - 1) / KCH;
    issue(As0, Bs0, 0);
    issue(As1, Bs1, KCH);
    __builtin_amdgcn_s_waitcnt(vm_lgkm0(DS::NI));  // chunk 0 loaded
    __builtin_amdgcn_s_barrier();
    issue(As2, Bs2, 2 * KCH);
    // chunk q in buffer q % 3: sum it, wait until chunk q + 1 has loaded (q + 2
    // in flight) and every wave is past its reads, then refill it with q + 3
    auto step = [&](uint32_t (*As)[TNV * KCH], uint32_t (*Bs)[TMV * KCH], int q) __attribute__((always_inline)) {
      compute(As, Bs);
      __builtin_amdgcn_s_waitcnt(vm_lgkm0(DS::NI));
      __builtin_amdgcn_s_barrier();
      issue(As, Bs, (q + 3) * KCH);
    };
    for (int q = 0; q < nch; q += 3) {
      step(As0, Bs0, q);
      if (q + 1 < nch) step(As1, Bs1, q + 1);
      if (q + 2 < nch) step(As2, Bs2, q + 2);
    }
    // no LDS write may be in flight when the workgroup ends
    __builtin_amdgcn_s_waitcnt(vm_lgkm0(0));
  }
  if (flags & kOutSplit)
    store_out_split<ADJ, RT, CT>(d, R, r0, n0, acc, wn, wm, out, ld_out, nrhs, scale);
  else
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
// split input state (k_stage_bf16x3_dma; the PF / DB flags are not used)
using D0 = Shape<256, 128, 512, 2, 4, true, true>;
using D1 = Shape<128, 128, 256, 2, 4, true, true>;
using D2 = Shape<128, 64, 256, 2, 2, true, true>;
using D3 = Shape<64, 64, 256, 1, 2, true, true>;

struct VariantDims {
  int tnv, tmv, nth;
};
template <class S>
constexpr VariantDims dims_of() {
  return {S::TNV, S::TMV, S::NTH};
}

VariantDims variant_dims(int prec, bool in_split, int v) {
  if (in_split) {
    switch (v) {
      case 0: return dims_of<D0>();
      case 1: return dims_of<D1>();
      case 2: return dims_of<D2>();
      default: return dims_of<D3>();
    }
  }
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
// Variant choice per (kernel family, direction, output-rows bucket, reduction
// bucket, RHS tiles); the family is the precision, plus 16 for the split-BF16
// kernels of split input states.  Filled by autotune_stage (timing every
// variant on the stage's real shape) and optionally persisted as text lines
// "family adj rb qb nb variant" in the file named by MBF_TUNE_FILE.
namespace {
using TuneKey = std::tuple<int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

constexpr int kSplitFamily = 16;
// Key family of the split-state choice (see split_choice).
constexpr int kSplitChoice = 64;
inline int family(int prec, bool in_split) { return prec + (in_split ? kSplitFamily : 0); }
inline int family_variants(int fam) {
  return fam >= kSplitFamily ? num_variants(fam - kSplitFamily, true) : num_variants(fam, false);
}

TuneKey tune_key(int prec, bool in_split, bool adj, int R, int Q, int nrhs) {
  return TuneKey{family(prec, in_split), adj ? 1 : 0, (R + 63) / 64, (Q + 63) / 64,
                 (nrhs + kTuneRhs - 1) / kTuneRhs};
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
    if ((a == MBF_C64 || a == MBF_C64_SPLIT_BF16 || a == MBF_C64_SPLIT_BF16 + kSplitFamily) && v >= 0 &&
        v < family_variants(a))
      g_tune[TuneKey{a, b, c, d, e}] = v;
    else if (a == kSplitChoice + MBF_C64_SPLIT_BF16 && (v == 0 || v == 1))
      g_tune[TuneKey{a, b, c, d, e}] = v;
  std::fclose(f);
}
}  // namespace

int tuned_variant(int prec, bool in_split, bool adj, int R, int Q, int nrhs) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(tune_key(prec, in_split, adj, R, Q, nrhs));
  if (it != g_tune.end()) return it->second;
  if (const char* e = std::getenv("MBF_STAGE_VARIANT")) {  // taken modulo the family's variant count
    const int v = std::atoi(e);
    if (v >= 0) return v % num_variants(prec, in_split);
  }
  // Untuned defaults: the small FP32 tile; for BF16 x3 the double-buffered
  // 256 x 128 tile when the right-hand sides fill it, the 128 x 64 one for
  // mid-size batches, the 64 x 64 one for small batches.
  if (prec == MBF_C64) return 0;
  if (in_split) return nrhs >= 192 ? 0 : nrhs > 64 ? 2 : 3;
  return nrhs >= 192 ? 5 : nrhs > 64 ? 4 : 0;
}

namespace {
TuneKey split_key(int prec, int64_t rows, int nrhs) {
  return TuneKey{kSplitChoice + prec, 0, (int)(rows >> 16), 0, (nrhs + kTuneRhs - 1) / kTuneRhs};
}
}  // namespace

int split_choice(int prec, int64_t rows, int nrhs) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(split_key(prec, rows, nrhs));
  return it == g_tune.end() ? -1 : it->second;
}

void set_split_choice(int prec, int64_t rows, int nrhs, bool on) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  const TuneKey k = split_key(prec, rows, nrhs);
  g_tune[k] = on ? 1 : 0;
  if (const char* path = std::getenv("MBF_TUNE_FILE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                   std::get<4>(k), on ? 1 : 0);
      std::fclose(f);
    }
  }
}

template <bool ADJ>
static void launch_variant(int prec, int v, dim3 grid, hipStream_t st, const BlockDesc* blk, const void* W,
                           const float2* x, int64_t ld_in, float2* y, int64_t ld_out, int nrhs, const float* scale,
                           int mtiles, int ntiles, int64_t total, int flags) {
#define MBF_LAUNCH(KER, WT, S)                                                                            \
  hipLaunchKernelGGL((KER<ADJ, S>), grid, dim3(S::NTH), 0, st, blk, reinterpret_cast<const WT*>(W), x, ld_in, \
                     y, ld_out, nrhs, scale, mtiles, ntiles, total, flags)
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
  } else if (flags & kInSplit) {
    switch (v) {
      case 0: MBF_LAUNCH(k_stage_bf16x3_dma, uint2, D0); break;
      case 1: MBF_LAUNCH(k_stage_bf16x3_dma, uint2, D1); break;
      case 2: MBF_LAUNCH(k_stage_bf16x3_dma, uint2, D2); break;
      default: MBF_LAUNCH(k_stage_bf16x3_dma, uint2, D3); break;
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
                        hipStream_t st, bool in_split, bool out_split, int force_variant) {
  const int Rmax = adj ? P.max_K[s] : P.max_M[s];
  const int Qmax = adj ? P.max_M[s] : P.max_K[s];
  if (prec != MBF_C64 && prec != MBF_C64_SPLIT_BF16) return {MBF_ERR_UNSUPPORTED, "no MFMA stage kernel"};
  if (nrhs < 1) return {MBF_ERR_INVALID_ARG, "MFMA stage: nrhs < 1"};
  if ((in_split || out_split) && prec != MBF_C64_SPLIT_BF16)
    return {MBF_ERR_INVALID_ARG, "MFMA stage: split state outside the split-BF16 precision"};
  // Offsets of the split-input kernel's LDS loads are 32-bit byte offsets
  // within the 64 state columns of a wave.
  if (in_split && ld_in >= ((int64_t)1 << 23)) return {MBF_ERR_UNSUPPORTED, "MFMA stage: split state too tall"};
  const int v = force_variant >= 0 ? force_variant : tuned_variant(prec, in_split, adj, Rmax, Qmax, nrhs);
  if (v < 0 || v >= num_variants(prec, in_split)) return {MBF_ERR_INVALID_ARG, "MFMA stage: no such variant"};
  const VariantDims vd = variant_dims(prec, in_split, v);
  const int mtiles = std::max(1, (Rmax + vd.tmv - 1) / vd.tmv);
  const int ntiles = (nrhs + vd.tnv - 1) / vd.tnv;
  const int64_t total = (int64_t)P.nblk[s] * mtiles * ntiles;
  const int64_t grid = (total + kXcd - 1) / kXcd * kXcd;
  if (grid > INT32_MAX) return {MBF_ERR_UNSUPPORTED, "stage grid too large"};
  const float2* x = reinterpret_cast<const float2*>(in);
  float2* y = reinterpret_cast<float2*>(out);
  const int flags = (in_split ? kInSplit : 0) | (out_split ? kOutSplit : 0);
  if (adj)
    launch_variant<true>(prec, v, dim3((unsigned)grid), st, blk, W, x, ld_in, y, ld_out, nrhs, scale, mtiles, ntiles,
                         total, flags);
  else
    launch_variant<false>(prec, v, dim3((unsigned)grid), st, blk, W, x, ld_in, y, ld_out, nrhs, scale, mtiles, ntiles,
                          total, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("stage launch: ") + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

}  // namespace mbf

namespace mbf {

Error autotune_stage(const DevPart& P, int s, int prec, bool in_split, bool adj, const BlockDesc* blk,
                     const void* W, const void* in, int64_t ld_in, void* out, int64_t ld_out, int nrhs,
                     hipStream_t st, int* chosen, float* best_ms) {
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
  // split-BF16 stages write a split state except the last one; time that
  const bool out_split = prec == MBF_C64_SPLIT_BF16;
  for (int v = 0; v < num_variants(prec, in_split) && err.st == MBF_OK; ++v) {
    err = launch_stage_mfma(P, s, prec, adj, blk, W, in, ld_in, out, ld_out, nrhs, nullptr, st, in_split, out_split,
                            v);
    if (err.st != MBF_OK) break;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 2 && err.st == MBF_OK; ++r)
      err = launch_stage_mfma(P, s, prec, adj, blk, W, in, ld_in, out, ld_out, nrhs, nullptr, st, in_split,
                              out_split, v);
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
    const TuneKey k = tune_key(prec, in_split, adj, Rmax, Qmax, nrhs);
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
