// Apply kernels of the butterfly factorization (eq. (gbf), right to left)
// and their launch sequence.  See device.h for the HBM layout.
//
//   leaf_project      y_B = F_B^* x[B]   (x gathered through the point index)
//                     forward: F = V^L on Omega leaves; adjoint: F = U^L on X leaves
//   stage             out = W_blk in  (forward)  /  out = W_blk^* in (adjoint),
//                     one W_blk per (A, B'); the M^h scaling diag(1/sigma) is
//                     applied in the epilogue of the stage that produces the
//                     middle-level state
//   leaf_reconstruct  x[A] (+)= F_A z_A  (scatter through the point index)
//   dense_center      u += K_C g[Omega_C]       (multiscale, eq. (f1))
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "stage_mfma.h"
#include "stage_r16.h"

namespace mbf {

template <typename T>
struct cx;
template <>
struct cx<float> {
  using t = float2;
};
template <>
struct cx<double> {
  using t = double2;
};

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ __forceinline__ void cfma(C& acc, C a, C b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}
template <typename C>
__device__ __forceinline__ C cconj(C a) {
  a.y = -a.y;
  return a;
}
template <typename C>
__device__ __forceinline__ C czero() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}

// Selects instead of an indexed load keep the descriptor in registers.
__device__ __forceinline__ int32_t group_row(const BlockDesc& d, int32_t i) {
  int32_t base = d.orow[0] - d.ms[0];
  base = i >= d.ms[1] ? d.orow[1] - d.ms[1] : base;
  base = i >= d.ms[2] ? d.orow[2] - d.ms[2] : base;
  base = i >= d.ms[3] ? d.orow[3] - d.ms[3] : base;
  return base + i;
}

// ------------------------------------------------------------------ stage
// Tile of 64 output rows x 32 right-hand sides per pass, 16-deep reduction
// chunks staged in LDS; each of the 256 threads owns 4 x 2 outputs.
template <typename T, bool ADJ>
__global__ __launch_bounds__(256) void k_stage(const BlockDesc* __restrict__ blk,
                                               const typename cx<T>::t* __restrict__ W,
                                               const typename cx<T>::t* __restrict__ in,
                                               int64_t ld_in, typename cx<T>::t* __restrict__ out,
                                               int64_t ld_out, int nrhs,
                                               const T* __restrict__ scale) {
  using C = typename cx<T>::t;
  constexpr int BM = 64, BN = 32, BK = 16;
  __shared__ C As[BK][BM + 1];
  __shared__ C Bs[BN][BK + 1];
  const BlockDesc d = blk[blockIdx.x];
  const int R = ADJ ? d.K : d.M;
  const int Q = ADJ ? d.M : d.K;
  const int n0 = blockIdx.y * BN;
  const C* Wb = W + d.w_off;
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  for (int r0 = 0; r0 < R; r0 += BM) {
    C acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = czero<C>();
    for (int q0 = 0; q0 < Q; q0 += BK) {
      for (int e = tid; e < BK * BM; e += 256) {
        int q, r;
        if (!ADJ) {
          r = e % BM;
          q = e / BM;
        } else {
          q = e % BK;
          r = e / BK;
        }
        const int gr = r0 + r, gq = q0 + q;
        C v = czero<C>();
        if (gr < R && gq < Q)
          v = ADJ ? cconj(Wb[(int64_t)gr * d.M + gq]) : Wb[(int64_t)gq * d.M + gr];
        As[q][r] = v;
      }
      for (int e = tid; e < BK * BN; e += 256) {
        const int q = e % BK, n = e / BK;
        const int gq = q0 + q, gn = n0 + n;
        C v = czero<C>();
        if (gq < Q && gn < nrhs) {
          const int32_t row = ADJ ? group_row(d, gq) : d.in_row + gq;
          v = in[(int64_t)gn * ld_in + row];
        }
        Bs[n][q] = v;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < BK; ++q) {
        C a[4], b[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[q][tr + 16 * i];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[tc + 16 * j][q];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) cfma(acc[i][j], a[i], b[j]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gr = r0 + tr + 16 * i, gn = n0 + tc + 16 * j;
        if (gr < R && gn < nrhs) {
          const int32_t row = ADJ ? d.in_row + gr : group_row(d, gr);
          C v = acc[i][j];
          if (scale) {
            const T s = scale[row];
            v.x *= s;
            v.y *= s;
          }
          out[(int64_t)gn * ld_out + row] = v;
        }
      }
  }
}

// ------------------------------------------------------------------ leaves
// out[row + k, n] = sum_i conj(F[i + k np]) x[idx[p_off + i], n]
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_project(const LeafDesc* __restrict__ leaves,
                                                      const typename cx<T>::t* __restrict__ F,
                                                      const int32_t* __restrict__ idx,
                                                      const typename cx<T>::t* __restrict__ x,
                                                      int64_t ldx, typename cx<T>::t* __restrict__ out,
                                                      int64_t ld_out, int nrhs,
                                                      const T* __restrict__ scale) {
  using C = typename cx<T>::t;
  __shared__ C Xs[64][33];
  __shared__ C Fs[64][65];
  const LeafDesc d = leaves[blockIdx.x];
  const int n0 = blockIdx.y * 32;
  const int tid = threadIdx.x;
  const int tk = tid & 63, tn = tid >> 6;
  const C* Fb = F + d.f_off;
  for (int k0 = 0; k0 < d.r; k0 += 64) {
    C acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = czero<C>();
    for (int i0 = 0; i0 < d.np; i0 += 64) {
      // branch-free: clamped addresses, all loads in flight, zeros selected at the LDS store
      const int i = tid & 63, ic = min(i0 + i, d.np - 1);
      const int64_t p = idx[d.p_off + ic];
      C xv[8], fv[16];
#pragma unroll
      for (int r = 0; r < 8; ++r) xv[r] = x[(int64_t)min(n0 + (tid >> 6) + 4 * r, nrhs - 1) * ldx + p];
#pragma unroll
      for (int r = 0; r < 16; ++r) fv[r] = Fb[(int64_t)min(k0 + (tid >> 6) + 4 * r, d.r - 1) * d.np + ic];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int n = (tid >> 6) + 4 * r;
        Xs[i][n] = (i0 + i < d.np && n0 + n < nrhs) ? xv[r] : czero<C>();
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int k = (tid >> 6) + 4 * r;
        Fs[i][k] = (i0 + i < d.np && k0 + k < d.r) ? cconj(fv[r]) : czero<C>();
      }
      __syncthreads();
      const int ilim = min(64, d.np - i0);
      for (int i = 0; i < ilim; ++i) {
        const C f = Fs[i][tk];
#pragma unroll
        for (int j = 0; j < 8; ++j) cfma(acc[j], f, Xs[i][tn + 4 * j]);
      }
      __syncthreads();
    }
    if (k0 + tk < d.r) {
      const int32_t row = d.row + k0 + tk;
      const T s = scale ? scale[row] : T(1);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = n0 + tn + 4 * j;
        if (n < nrhs) {
          C v = acc[j];
          v.x *= s;
          v.y *= s;
          out[(int64_t)n * ld_out + row] = v;
        }
      }
    }
  }
}

// x[idx[p_off + i], n] (+)= sum_k F[i + k np] z[row + k, n]
// One workgroup per (leaf, chunk of 64 points, 32 right-hand sides): the rows
// of a leaf are independent, so large leaves (the coarse coronas of the
// multiscale split have leaves of thousands of points) spread over many
// workgroups.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_reconstruct(const LeafDesc* __restrict__ leaves,
                                                          const typename cx<T>::t* __restrict__ F,
                                                          const int32_t* __restrict__ idx,
                                                          const typename cx<T>::t* __restrict__ z,
                                                          int64_t ldz, typename cx<T>::t* __restrict__ x,
                                                          int64_t ldx, int nrhs, int accumulate) {
  using C = typename cx<T>::t;
  __shared__ C Zs[64][33];
  const LeafDesc d = leaves[blockIdx.x];
  const int i0 = blockIdx.y * 64;
  if (i0 >= d.np) return;
  const int n0 = blockIdx.z * 32;
  const int tid = threadIdx.x;
  const int ti = tid & 63, tn = tid >> 6;
  const C* Fb = F + d.f_off;
  C acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = czero<C>();
  // Branch-free loads (clamped addresses): the Z slab's loads are issued
  // together, and F is read 8 reduction entries at a time; rows of Zs past
  // the rank are zero, so the last group of 8 needs no guard.  Lanes past the
  // leaf's last point compute on a clamped point and are not stored.
  const int ic = min(i0 + ti, d.np - 1);
  for (int k0 = 0; k0 < d.r; k0 += 64) {
    C zv[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      zv[r] = z[(int64_t)min(n0 + tn + 4 * r, nrhs - 1) * ldz + d.row + min(k0 + ti, d.r - 1)];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int n = tn + 4 * r;
      Zs[ti][n] = (k0 + ti < d.r && n0 + n < nrhs) ? zv[r] : czero<C>();
    }
    __syncthreads();
    const int klim = min(64, d.r - k0);
    for (int k = 0; k < klim; k += 8) {
      C f[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) f[u] = Fb[(int64_t)min(k0 + k + u, d.r - 1) * d.np + ic];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int j = 0; j < 8; ++j) cfma(acc[j], f[u], Zs[k + u][tn + 4 * j]);
    }
    __syncthreads();
  }
  if (i0 + ti < d.np) {
    const int64_t p = idx[d.p_off + i0 + ti];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = n0 + tn + 4 * j;
      if (n < nrhs) {
        C v = acc[j];
        C* o = x + (int64_t)n * ldx + p;
        if (accumulate) {
          C w = *o;
          v.x += w.x;
          v.y += w.y;
        }
        *o = v;
      }
    }
  }
}

// Projection onto leaves with many points (the coarse coronas of the
// multiscale split, up to all N points in one leaf), in two passes.  Pass 1:
// one wave per (leaf, segment of seg points, KRW output rows, 16 right-hand
// sides); the lanes stride over the segment's points, every gathered state
// entry serves the wave's KRW rows, and the sums are combined across the wave
// with shuffles into part[((leaf maxseg + segment) nrhs + n) max_r + k].
// Pass 2 adds a leaf's segments in order (deterministic) and scales.  With
// one segment per leaf (part null) pass 1 scales and stores the sums itself.
template <typename T>
constexpr int wide_rows() {  // output rows per wave (KRW): 4 in FP32, 2 in FP64 (registers)
  return sizeof(T) == 4 ? 4 : 2;
}
constexpr int kWideSeg = 1024;  // points per segment

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_project_wide(const LeafDesc* __restrict__ leaves,
                                                           const typename cx<T>::t* __restrict__ F,
                                                           const int32_t* __restrict__ idx,
                                                           const typename cx<T>::t* __restrict__ x,
                                                           int64_t ldx, typename cx<T>::t* __restrict__ part,
                                                           typename cx<T>::t* __restrict__ out, int64_t ld_out,
                                                           const T* __restrict__ scale, int nrhs, int seg,
                                                           int maxseg, int max_r) {
  using C = typename cx<T>::t;
  constexpr int NRW = 16, KRW = wide_rows<T>();
  const int leaf = blockIdx.x / maxseg, sg = blockIdx.x % maxseg;
  const LeafDesc d = leaves[leaf];
  const int p_lo = sg * seg, p_hi = min(d.np, p_lo + seg);
  const int k0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * KRW;
  if (p_lo >= d.np || k0 >= d.r) return;  // whole wave; no workgroup barrier below
  const int lane = threadIdx.x & 63;
  const int n0 = blockIdx.z * NRW;
  const int nn = min(NRW, nrhs - n0);
  C acc[KRW][NRW];
#pragma unroll
  for (int j = 0; j < KRW; ++j)
#pragma unroll
    for (int n = 0; n < NRW; ++n) acc[j][n] = czero<C>();
  // The NRW loads of a point are issued together (right-hand sides past nrhs
  // read the last one again, rows past r read row r - 1; neither is stored):
  // a guarded load would wait for its data before the next one is issued.
#pragma unroll 2
  for (int i = p_lo + lane; i < p_hi; i += 64) {
    C f[KRW];
#pragma unroll
    for (int j = 0; j < KRW; ++j) f[j] = cconj(F[d.f_off + (int64_t)min(k0 + j, d.r - 1) * d.np + i]);
    const int64_t p = idx[d.p_off + i];
    C xv[NRW];
#pragma unroll
    for (int n = 0; n < NRW; ++n) xv[n] = x[(int64_t)min(n0 + n, nrhs - 1) * ldx + p];
#pragma unroll
    for (int j = 0; j < KRW; ++j)
#pragma unroll
      for (int n = 0; n < NRW; ++n) cfma(acc[j][n], f[j], xv[n]);
  }
#pragma unroll
  for (int j = 0; j < KRW; ++j)
#pragma unroll
    for (int n = 0; n < NRW; ++n)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        acc[j][n].x += __shfl_xor(acc[j][n].x, off);
        acc[j][n].y += __shfl_xor(acc[j][n].y, off);
      }
  // lane j NRW + n stores (row k0 + j, right-hand side n0 + n)
  C* pb = part ? part + (int64_t)blockIdx.x * nrhs * max_r : nullptr;
#pragma unroll
  for (int j = 0; j < KRW; ++j)
#pragma unroll
    for (int n = 0; n < NRW; ++n)
      if (lane == j * NRW + n && n < nn && k0 + j < d.r) {
        if (pb) {
          pb[(int64_t)(n0 + n) * max_r + k0 + j] = acc[j][n];
        } else {
          const int32_t row = d.row + k0 + j;
          const T sc = scale ? scale[row] : T(1);
          C v = acc[j][n];
          v.x *= sc;
          v.y *= sc;
          out[(int64_t)(n0 + n) * ld_out + row] = v;
        }
      }
}

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_project_wide_sum(const LeafDesc* __restrict__ leaves,
                                                               const typename cx<T>::t* __restrict__ part,
                                                               typename cx<T>::t* __restrict__ out,
                                                               int64_t ld_out, int nrhs, int seg, int maxseg,
                                                               int max_r, const T* __restrict__ scale) {
  using C = typename cx<T>::t;
  const LeafDesc d = leaves[blockIdx.x];
  const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int k = (int)(e % max_r), n = (int)(e / max_r);
  if (n >= nrhs || k >= d.r) return;
  const int nseg = (d.np + seg - 1) / seg;
  const C* pb = part + ((int64_t)blockIdx.x * maxseg * nrhs + n) * max_r + k;
  // the segment loads are independent: unrolled, they are in flight together
  C v = czero<C>();
#pragma unroll 8
  for (int sg = 0; sg < nseg; ++sg) {
    const C a = pb[(int64_t)sg * nrhs * max_r];
    v.x += a.x;
    v.y += a.y;
  }
  const int32_t row = d.row + k;
  const T sc = scale ? scale[row] : T(1);
  v.x *= sc;
  v.y *= sc;
  out[(int64_t)n * ld_out + row] = v;
}

// Small leaves (at most 16 points and rank 16, e.g. 4 x 4 leaves): one
// workgroup per leaf and 64 right-hand sides; thread (t % 16, t / 16) owns
// output row t % 16 for the right-hand sides t / 16 + 16 j.  The stores of 16
// consecutive lanes cover 16 consecutive state rows (projection) or the
// leaf's gathered points (reconstruction).
constexpr int kSmallLeaf = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_project_small(const LeafDesc* __restrict__ leaves,
                                                            const typename cx<T>::t* __restrict__ F,
                                                            const int32_t* __restrict__ idx,
                                                            const typename cx<T>::t* __restrict__ x,
                                                            int64_t ldx, typename cx<T>::t* __restrict__ out,
                                                            int64_t ld_out, int nrhs,
                                                            const T* __restrict__ scale) {
  using C = typename cx<T>::t;
  __shared__ C Xs[kSmallLeaf][65];
  __shared__ C Fs[kSmallLeaf][kSmallLeaf + 1];
  const LeafDesc d = leaves[blockIdx.x];
  const int n0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const C* Fb = F + d.f_off;
  for (int e = tid; e < kSmallLeaf * 64; e += 256) {
    const int i = e & 15, n = e >> 4;
    C v = czero<C>();
    if (i < d.np && n0 + n < nrhs) v = x[(int64_t)(n0 + n) * ldx + idx[d.p_off + i]];
    Xs[i][n] = v;
  }
  {
    const int i = tid & 15, k = tid >> 4;
    C v = czero<C>();
    if (i < d.np && k < d.r) v = cconj(Fb[(int64_t)k * d.np + i]);
    Fs[i][k] = v;
  }
  __syncthreads();
  const int tk = tid & 15, tn = tid >> 4;
  C acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = czero<C>();
  for (int i = 0; i < d.np; ++i) {
    const C f = Fs[i][tk];
#pragma unroll
    for (int j = 0; j < 4; ++j) cfma(acc[j], f, Xs[i][tn + 16 * j]);
  }
  if (tk < d.r) {
    const int32_t row = d.row + tk;
    const T s = scale ? scale[row] : T(1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tn + 16 * j;
      if (n < nrhs) {
        C v = acc[j];
        v.x *= s;
        v.y *= s;
        out[(int64_t)n * ld_out + row] = v;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_reconstruct_small(const LeafDesc* __restrict__ leaves,
                                                                const typename cx<T>::t* __restrict__ F,
                                                                const int32_t* __restrict__ idx,
                                                                const typename cx<T>::t* __restrict__ z,
                                                                int64_t ldz, typename cx<T>::t* __restrict__ x,
                                                                int64_t ldx, int nrhs, int accumulate) {
  using C = typename cx<T>::t;
  __shared__ C Zs[kSmallLeaf][65];
  __shared__ C Fs[kSmallLeaf][kSmallLeaf + 1];
  const LeafDesc d = leaves[blockIdx.x];
  const int n0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const C* Fb = F + d.f_off;
  for (int e = tid; e < kSmallLeaf * 64; e += 256) {
    const int k = e & 15, n = e >> 4;
    C v = czero<C>();
    if (k < d.r && n0 + n < nrhs) v = z[(int64_t)(n0 + n) * ldz + d.row + k];
    Zs[k][n] = v;
  }
  {
    const int i = tid & 15, k = tid >> 4;
    C v = czero<C>();
    if (i < d.np && k < d.r) v = Fb[(int64_t)k * d.np + i];
    Fs[i][k] = v;
  }
  __syncthreads();
  const int ti = tid & 15, tn = tid >> 4;
  if (ti >= d.np) return;
  C acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = czero<C>();
  for (int k = 0; k < d.r; ++k) {
    const C f = Fs[ti][k];
#pragma unroll
    for (int j = 0; j < 4; ++j) cfma(acc[j], f, Zs[k][tn + 16 * j]);
  }
  const int64_t p = idx[d.p_off + ti];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + tn + 16 * j;
    if (n < nrhs) {
      C v = acc[j];
      C* o = x + (int64_t)n * ldx + p;
      if (accumulate) {
        const C w = *o;
        v.x += w.x;
        v.y += w.y;
      }
      *o = v;
    }
  }
}

// u[i, n] (+)= sum_k KC[i + k nx] g[cidx[k], n]     (dense center, forward)
template <typename T>
__global__ __launch_bounds__(256) void k_center_fwd(const typename cx<T>::t* __restrict__ KC,
                                                    const int32_t* __restrict__ cidx, int64_t nx,
                                                    int32_t nc, const typename cx<T>::t* __restrict__ g,
                                                    int64_t ldg, typename cx<T>::t* __restrict__ u,
                                                    int64_t ldu, int nrhs, int accumulate) {
  using C = typename cx<T>::t;
  __shared__ C Gs[64][33];
  const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int tn = threadIdx.x >> 6;
  const int n0 = blockIdx.y * 32;
  C acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = czero<C>();
  for (int k0 = 0; k0 < nc; k0 += 64) {
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int k = e & 63, n = e >> 6;
      C v = czero<C>();
      if (k0 + k < nc && n0 + n < nrhs) v = g[(int64_t)(n0 + n) * ldg + cidx[k0 + k]];
      Gs[k][n] = v;
    }
    __syncthreads();
    if (i < nx) {
      const int klim = min(64, nc - k0);
      for (int k = 0; k < klim; ++k) {
        const C f = KC[(int64_t)(k0 + k) * nx + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) cfma(acc[j], f, Gs[k][tn + 4 * j]);
      }
    }
    __syncthreads();
  }
  if (i < nx) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = n0 + tn + 4 * j;
      if (n < nrhs) {
        C v = acc[j];
        C* o = u + (int64_t)n * ldu + i;
        if (accumulate) {
          C w = *o;
          v.x += w.x;
          v.y += w.y;
        }
        *o = v;
      }
    }
  }
}

// Adjoint of the dense center, pass 1: partial[chunk, n, k] = sum over the
// chunk's rows i of conj(KC[i + k nx]) h[i, n].  One workgroup per (chunk of
// rows, 64 center columns k, 16 right-hand sides).  The chunk is walked in
// slabs of 64 rows staged in LDS, loaded along the rows (the contiguous index
// of both KC and h; addresses clamped into range, zeros selected at the
// LDS store); thread (k = tid % 64, group g = tid / 64) sums right-hand sides
// 4 g .. 4 g + 3, reading KC from its LDS row and h as a broadcast.
template <typename T>
__global__ __launch_bounds__(256) void k_center_adj_partial(const typename cx<T>::t* __restrict__ KC,
                                                            int64_t nx, int32_t nc,
                                                            const typename cx<T>::t* __restrict__ h,
                                                            int64_t ldh, int nrhs, int64_t chunk_rows,
                                                            typename cx<T>::t* __restrict__ part) {
  using C = typename cx<T>::t;
  __shared__ C Ks[64][65];  // [k][i], conj(KC)
  __shared__ C Hs[64][17];  // [i][n]
  const int tid = threadIdx.x, kk = tid & 63, g = tid >> 6;
  const int k0 = blockIdx.y * 64, n0 = blockIdx.z * 16;
  const int64_t i0 = (int64_t)blockIdx.x * chunk_rows, i1 = min(i0 + chunk_rows, nx);
  C acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = czero<C>();
  for (int64_t sl = i0; sl < i1; sl += 64) {
    C kv[16], hv[4];
#pragma unroll
    for (int r = 0; r < 16; ++r) {  // KC slab: 64 k x 64 rows, lanes along the rows
      const int e = tid + 256 * r, k = e >> 6, i = e & 63;
      kv[r] = KC[(int64_t)min(k0 + k, nc - 1) * nx + min(sl + i, i1 - 1)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // h slab: 64 rows x 16 RHS
      const int e = tid + 256 * r, n = e >> 6, i = e & 63;
      hv[r] = h[(int64_t)min(n0 + n, nrhs - 1) * ldh + min(sl + i, i1 - 1)];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = tid + 256 * r, k = e >> 6, i = e & 63;
      Ks[k][i] = (k0 + k < nc && sl + i < i1) ? cconj(kv[r]) : czero<C>();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r, n = e >> 6, i = e & 63;
      Hs[i][n] = (n0 + n < nrhs && sl + i < i1) ? hv[r] : czero<C>();
    }
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < 64; ++i) {
      const C f = Ks[kk][i];
#pragma unroll
      for (int j = 0; j < 4; ++j) cfma(acc[j], f, Hs[i][4 * g + j]);
    }
    __syncthreads();
  }
  if (k0 + kk < nc) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + 4 * g + j;
      if (n < nrhs) part[((int64_t)blockIdx.x * nrhs + n) * nc + k0 + kk] = acc[j];
    }
  }
}

// Pass 2: v[cidx[k], n] = sum over chunks of partial[chunk, k, n].
template <typename T>
__global__ __launch_bounds__(256) void k_center_adj_reduce(const typename cx<T>::t* __restrict__ part,
                                                           int nchunk, int32_t nc,
                                                           const int32_t* __restrict__ cidx,
                                                           typename cx<T>::t* __restrict__ v,
                                                           int64_t ldv, int nrhs) {
  using C = typename cx<T>::t;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nc * nrhs) return;
  const int k = (int)(e % nc), n = (int)(e / nc);
  C s = czero<C>();
  for (int c = 0; c < nchunk; ++c) {
    const C p = part[((int64_t)c * nrhs + n) * nc + k];
    s.x += p.x;
    s.y += p.y;
  }
  v[(int64_t)n * ldv + cidx[k]] = s;
}

// ------------------------------------------------------------------ launch
namespace {

constexpr int kTN = 32;  // RHS per workgroup in the generic kernels

inline Error hip_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)};
  return {MBF_OK, ""};
}

inline unsigned ntiles(int64_t nrhs) { return (unsigned)((nrhs + kTN - 1) / kTN); }

// Event pair around one launch when profiling is active.
struct Timed {
  Profiler* pr;
  hipStream_t st;
  int idx = -1;
  Timed(Profiler* p, hipStream_t s, int kind, int part, int stage, int prec, double flops, double bytes)
      : pr(p), st(s) {
    if (!pr || !pr->on || pr->used >= pr->cap) return;
    idx = pr->used++;
    pr->rec[idx] = mbf_launch_record{kind, part, stage, prec, 0.0, flops, bytes};
    (void)hipEventRecord(pr->ev[2 * idx], st);
  }
  ~Timed() {
    if (idx >= 0) (void)hipEventRecord(pr->ev[2 * idx + 1], st);
  }
};

inline int64_t stage_nnz(const DevPart& P, int s) {
  const int64_t e = (s + 1 < P.L) ? P.w_stage_off[s + 1] : P.w_elems;
  return e - P.w_stage_off[s];
}

// States between the split-BF16 stages: MBF_BF16_SPLIT_STATE=0 keeps them
// FP32 (every stage then splits its input as it stages it through LDS), =1
// keeps them split whatever the autotuner chose; unset, the autotuner's
// choice decides (split when it has not timed the factorization).
int split_state_mode() {
  const char* e = std::getenv("MBF_BF16_SPLIT_STATE");
  if (!e || !e[0]) return -1;
  return e[0] == '0' ? 0 : 1;
}

// One part of the apply on stream st.  ws holds its two state buffers of
// buf_ld x nrhs entries each; ws_ld (the widest state of the factorization)
// keys the split-BF16 state choice.  Forward: the leaf reconstruction, which
// writes or adds into `out`, waits for `before_out` and records `after_out`
// (either may be null), so that the parts of a multiscale sum add into u in
// a fixed order while the rest of their work overlaps.
template <typename T>
Error run_part(const DevPart& P, int pidx, Profiler* pr, int prec, bool adj, int64_t nrhs, const void* in,
               int64_t ldin, void* out, int64_t ldout, void* ws, int64_t ws_ld, int64_t buf_ld, bool accumulate,
               hipStream_t st, hipEvent_t before_out = nullptr, hipEvent_t after_out = nullptr) {
  using C = typename cx<T>::t;
  const PrecData& pd = P.prec[prec];
  C* buf[2] = {reinterpret_cast<C*>(ws), reinterpret_cast<C*>(ws) + buf_ld * nrhs};
  const T* S = reinterpret_cast<const T*>(pd.S);
  const int L = P.L, m = P.m;
  const unsigned nt = ntiles(nrhs);
  const int ni = (int)nrhs;
  const double es = sizeof(C), ef = (prec == MBF_C128) ? 16.0 : 8.0, nr = (double)nrhs;
  auto stage_cost = [&](int s, double& fl, double& by) {
    const double z = (double)stage_nnz(P, s);
    fl = 8.0 * z * nr;
    by = z * ef + (double)(P.rows[s] + P.rows[s + 1]) * nr * es;
  };
  const C* Vf = reinterpret_cast<const C*>(pd.V0);
  const C* Uf = reinterpret_cast<const C*>(pd.UL);
  const bool v_small = P.max_vnp <= kSmallLeaf && P.max_vr <= kSmallLeaf;
  const bool u_small = P.max_unp <= kSmallLeaf && P.max_ur <= kSmallLeaf;
  const unsigned nt64 = (unsigned)((nrhs + 63) / 64);
  // part: the other state buffer (ws_ld x nrhs entries), free during the projection
  auto project = [&](bool small, int32_t nleaf, int32_t max_np, int32_t max_r, const LeafDesc* lv, const C* Fl,
                     const int32_t* idx, C* dst, int64_t lddst, const T* sc, C* part) {
    if (!small && max_np > 256) {
      // segments of kWideSeg points when their partial sums fit the buffer,
      // else one segment per leaf, summed in place
      int seg = kWideSeg, maxseg = (max_np + kWideSeg - 1) / kWideSeg;
      const bool two = maxseg > 1 && (int64_t)nleaf * maxseg * max_r <= buf_ld;
      if (!two) seg = max_np, maxseg = 1;
      hipLaunchKernelGGL(k_leaf_project_wide<T>,
                         dim3((unsigned)(nleaf * maxseg),
                              (unsigned)((max_r + 4 * wide_rows<T>() - 1) / (4 * wide_rows<T>())),
                              (unsigned)((nrhs + 15) / 16)),
                         dim3(256), 0, st, lv, Fl, idx, reinterpret_cast<const C*>(in), ldin, two ? part : nullptr,
                         dst, lddst, sc, ni, seg, maxseg, max_r);
      if (two)
        hipLaunchKernelGGL(k_leaf_project_wide_sum<T>,
                           dim3(nleaf, (unsigned)(((int64_t)max_r * nrhs + 255) / 256)), dim3(256), 0, st, lv, part,
                           dst, lddst, ni, seg, maxseg, max_r, sc);
    } else if (small)
      hipLaunchKernelGGL(k_leaf_project_small<T>, dim3(nleaf, nt64), dim3(256), 0, st, lv, Fl, idx,
                         reinterpret_cast<const C*>(in), ldin, dst, lddst, ni, sc);
    else
      hipLaunchKernelGGL(k_leaf_project<T>, dim3(nleaf, nt), dim3(256), 0, st, lv, Fl, idx,
                         reinterpret_cast<const C*>(in), ldin, dst, lddst, ni, sc);
  };
  // Split BF16: the stage kernels pass the state between stages as BF16
  // hi | lo words; the first stage splits the projected FP32 state, the last
  // one writes FP32 for the leaf reconstruction.
  const int mode = split_state_mode();
  const bool split = prec == MBF_C64_SPLIT_BF16 && ws_ld < ((int64_t)1 << 23) &&
                     (mode == 1 || (mode == -1 && split_choice(prec, ws_ld, ni) != 0));
  int s_lo = L, s_hi = -1;  // first and last stage with blocks
  for (int s = 0; s < L; ++s)
    if (P.nblk[s] > 0) {
      s_lo = std::min(s_lo, s);
      s_hi = s;
    }
  auto reconstruct = [&](bool small, int32_t nleaf, int32_t max_np, const LeafDesc* lv, const C* Fl,
                         const int32_t* idx, const C* src, int64_t ldsrc, int acc) {
    if (small)
      hipLaunchKernelGGL(k_leaf_reconstruct_small<T>, dim3(nleaf, nt64), dim3(256), 0, st, lv, Fl, idx, src, ldsrc,
                         reinterpret_cast<C*>(out), ldout, ni, acc);
    else
      hipLaunchKernelGGL(k_leaf_reconstruct<T>, dim3(nleaf, (unsigned)((max_np + 63) / 64), nt), dim3(256), 0, st,
                         lv, Fl, idx, src, ldsrc, reinterpret_cast<C*>(out), ldout, ni, acc);
  };
  if (!adj) {
    if (P.n_vleaf > 0) {
      Timed t(pr, st, 0, pidx, 0, prec, 8.0 * P.v_elems * nr, P.v_elems * es + (P.nxi + P.rows[0]) * nr * es);
      project(v_small, P.n_vleaf, P.max_vnp, P.max_vr, P.d_vleaf, Vf, P.d_vidx, buf[0], P.ld[0], m == 0 ? S : nullptr,
              buf[1]);
    }
    for (int s = 0; s < L; ++s) {
      if (P.nblk[s] == 0) continue;
      const T* sc = (s == m - 1) ? S : nullptr;
      const BlockDesc* bd = P.d_blk + P.blk_first[s];
      double fl, by;
      stage_cost(s, fl, by);
      Timed t(pr, st, 1, pidx, s, prec, fl, by);
      if (prec != MBF_C128 && use_mfma(P, s, nrhs, prec)) {
        Error e = launch_stage_mfma(P, s, prec, false, bd, pd.Wst[s], buf[s & 1], P.ld[s], buf[(s + 1) & 1],
                                    P.ld[s + 1], ni, reinterpret_cast<const float*>(sc), st, split && s != s_lo,
                                    split && s != s_hi);
        if (e.st != MBF_OK) return e;
      } else if (prec == MBF_C64) {
        Error e = launch_stage_r16(P, s, false, bd, pd.Wst[s], buf[s & 1], P.ld[s], buf[(s + 1) & 1], P.ld[s + 1], ni,
                                   reinterpret_cast<const float*>(sc), st);
        if (e.st != MBF_OK) return e;
      } else {
        hipLaunchKernelGGL((k_stage<T, false>), dim3(P.nblk[s], nt), dim3(256), 0, st, bd,
                           reinterpret_cast<const C*>(pd.Wst[s]), buf[s & 1],
                           P.ld[s], buf[(s + 1) & 1], P.ld[s + 1], ni, sc);
      }
    }
    if (before_out && hipStreamWaitEvent(st, before_out, 0) != hipSuccess) return {MBF_ERR_HIP, "hipStreamWaitEvent"};
    if (P.n_uleaf > 0) {
      Timed t(pr, st, 2, pidx, L, prec, 8.0 * P.u_elems * nr, P.u_elems * es + (P.nx + P.rows[L]) * nr * es);
      reconstruct(u_small, P.n_uleaf, P.max_unp, P.d_uleaf, Uf, P.d_uidx, buf[L & 1], P.ld[L], accumulate ? 1 : 0);
    }
    if (after_out && hipEventRecord(after_out, st) != hipSuccess) return {MBF_ERR_HIP, "hipEventRecord"};
  } else {
    if (P.n_uleaf > 0) {
      Timed t(pr, st, 0, pidx, L, prec, 8.0 * P.u_elems * nr, P.u_elems * es + (P.nx + P.rows[L]) * nr * es);
      project(u_small, P.n_uleaf, P.max_unp, P.max_ur, P.d_uleaf, Uf, P.d_uidx, buf[L & 1], P.ld[L],
              m == L ? S : nullptr, buf[(L + 1) & 1]);
    }
    for (int s = L - 1; s >= 0; --s) {
      if (P.nblk[s] == 0) continue;
      const T* sc = (s == m) ? S : nullptr;
      const BlockDesc* bd = P.d_blk + P.blk_first[s];
      double fl, by;
      stage_cost(s, fl, by);
      Timed t(pr, st, 1, pidx, s, prec, fl, by);
      if (prec != MBF_C128 && use_mfma(P, s, nrhs, prec)) {
        Error e = launch_stage_mfma(P, s, prec, true, bd, pd.Wst[s], buf[(s + 1) & 1], P.ld[s + 1], buf[s & 1],
                                    P.ld[s], ni, reinterpret_cast<const float*>(sc), st, split && s != s_hi,
                                    split && s != s_lo);
        if (e.st != MBF_OK) return e;
      } else if (prec == MBF_C64) {
        Error e = launch_stage_r16(P, s, true, bd, pd.Wst[s], buf[(s + 1) & 1], P.ld[s + 1], buf[s & 1], P.ld[s], ni,
                                   reinterpret_cast<const float*>(sc), st);
        if (e.st != MBF_OK) return e;
      } else {
        hipLaunchKernelGGL((k_stage<T, true>), dim3(P.nblk[s], nt), dim3(256), 0, st, bd,
                           reinterpret_cast<const C*>(pd.Wst[s]), buf[(s + 1) & 1],
                           P.ld[s + 1], buf[s & 1], P.ld[s], ni, sc);
      }
    }
    if (P.n_vleaf > 0) {
      Timed t(pr, st, 2, pidx, 0, prec, 8.0 * P.v_elems * nr, P.v_elems * es + (P.nxi + P.rows[0]) * nr * es);
      reconstruct(v_small, P.n_vleaf, P.max_vnp, P.d_vleaf, Vf, P.d_vidx, buf[0], P.ld[0], 0);
    }
  }
  return hip_check("apply launch");
}

// Rows per chunk of the center adjoint's first pass: at least 512, and at most
// 128 chunks (the partial sums take chunks x n_center x nrhs entries).
inline int64_t center_chunk_rows(int64_t nx) {
  const int64_t per = (nx + 127) / 128;
  return std::max<int64_t>(512, (per + 63) / 64 * 64);
}

template <typename T>
Error run_center(const DevFactor& F, int prec, bool adj, int64_t nrhs, const void* in, int64_t ldin,
                 void* out, int64_t ldout, void* ws, bool accumulate, hipStream_t st) {
  using C = typename cx<T>::t;
  const C* KC = reinterpret_cast<const C*>(F.center[prec].center);
  const int32_t nc = (int32_t)F.n_center;
  const int ni = (int)nrhs;
  const double es = sizeof(C), nr = (double)nrhs, z = (double)F.nx * nc;
  Timed t(&F.prof, st, 3, -1, 0, prec, 8.0 * z * nr, z * es + (double)(F.nx + nc) * nr * es);
  if (!adj) {
    hipLaunchKernelGGL(k_center_fwd<T>, dim3((unsigned)((F.nx + 63) / 64), ntiles(nrhs)), dim3(256), 0,
                       st, KC, F.d_center_idx, F.nx, nc, reinterpret_cast<const C*>(in), ldin,
                       reinterpret_cast<C*>(out), ldout, ni, accumulate ? 1 : 0);
  } else {
    const int64_t ch = center_chunk_rows(F.nx);
    const int nchunk = (int)((F.nx + ch - 1) / ch);
    C* part = reinterpret_cast<C*>(ws);
    hipLaunchKernelGGL(k_center_adj_partial<T>, dim3(nchunk, (nc + 63) / 64, (unsigned)((nrhs + 15) / 16)),
                       dim3(256), 0, st, KC, F.nx, nc, reinterpret_cast<const C*>(in), ldin, ni, ch, part);
    hipLaunchKernelGGL(k_center_adj_reduce<T>, dim3((unsigned)(((int64_t)nc * nrhs + 255) / 256)),
                       dim3(256), 0, st, part, nchunk, nc, F.d_center_idx, reinterpret_cast<C*>(out),
                       ldout, ni);
  }
  return hip_check("center launch");
}

int64_t state_ld_max(const DevFactor& F) {
  int64_t mx = 4;
  for (auto& P : F.parts)
    for (auto v : P.ld) mx = std::max(mx, v);
  return mx;
}

}  // namespace

Error autotune_factor(const DevFactor& F, int prec, int64_t nrhs, void* ws, size_t ws_bytes, hipStream_t st,
                      int* ntuned) {
  if (ws_bytes < workspace_bytes(F, prec, nrhs)) return {MBF_ERR_INVALID_ARG, "workspace too small"};
  if (ntuned) *ntuned = 0;
  if (prec == MBF_C128) return {MBF_OK, ""};
  const int64_t ws_ld = state_ld_max(F);
  if (hipMemsetAsync(ws, 0, 2 * (size_t)ws_ld * nrhs * 8, st) != hipSuccess) return {MBF_ERR_HIP, "memset"};
  for (const auto& P : F.parts) {
    char* b0 = reinterpret_cast<char*>(ws);
    char* b1 = b0 + (size_t)ws_ld * nrhs * 8;
    char* buf[2] = {b0, b1};
    for (int s = 0; s < P.L; ++s) {
      if (P.nblk[s] == 0 || !use_mfma(P, s, nrhs, prec)) continue;
      const BlockDesc* bd = P.d_blk + P.blk_first[s];
      // split BF16: the kernels of FP32 inputs (first stage) and of split inputs
      for (int fam = 0; fam < (prec == MBF_C64_SPLIT_BF16 ? 2 : 1); ++fam)
        for (int adj = 0; adj < 2; ++adj) {
          Error e = adj ? autotune_stage(P, s, prec, fam == 1, true, bd, P.prec[prec].Wst[s], buf[(s + 1) & 1],
                                         P.ld[s + 1], buf[s & 1], P.ld[s], (int)nrhs, st, nullptr, nullptr)
                        : autotune_stage(P, s, prec, fam == 1, false, bd, P.prec[prec].Wst[s], buf[s & 1],
                                         P.ld[s], buf[(s + 1) & 1], P.ld[s + 1], (int)nrhs, st, nullptr, nullptr);
          if (e.st != MBF_OK) return e;
          if (ntuned) ++*ntuned;
        }
    }
  }
  if (prec == MBF_C64_SPLIT_BF16 && ws_ld < ((int64_t)1 << 23)) {
    // split or FP32 states between the stages: time both forward stage chains
    char* b0 = reinterpret_cast<char*>(ws);
    char* buf[2] = {b0, b0 + (size_t)ws_ld * nrhs * 8};
    auto chain = [&](bool on) -> Error {
      for (const auto& P : F.parts) {
        int s_lo = P.L, s_hi = -1;
        for (int s = 0; s < P.L; ++s)
          if (P.nblk[s] > 0) s_lo = std::min(s_lo, s), s_hi = s;
        for (int s = 0; s < P.L; ++s) {
          if (P.nblk[s] == 0) continue;
          Error e = launch_stage_mfma(P, s, prec, false, P.d_blk + P.blk_first[s], P.prec[prec].Wst[s], buf[s & 1],
                                      P.ld[s], buf[(s + 1) & 1], P.ld[s + 1], (int)nrhs, nullptr, st,
                                      on && s != s_lo, on && s != s_hi);
          if (e.st != MBF_OK) return e;
        }
      }
      return {MBF_OK, ""};
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return {MBF_ERR_HIP, "hipEventCreate"};
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return {MBF_ERR_HIP, "hipEventCreate"};
    }
    float ms[2] = {0.f, 0.f};
    Error err{MBF_OK, ""};
    for (int on = 0; on < 2 && err.st == MBF_OK; ++on) {
      err = chain(on == 1);  // warm-up
      if (err.st != MBF_OK) break;
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 2 && err.st == MBF_OK; ++r) err = chain(on == 1);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) err = {MBF_ERR_HIP, "autotune timing"};
      else (void)hipEventElapsedTime(&ms[on], e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err.st != MBF_OK) return err;
    set_split_choice(prec, ws_ld, (int)nrhs, ms[1] <= ms[0]);
  }
  return {MBF_OK, ""};
}

namespace {
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int64_t part_ld_max(const DevPart& P) {
  int64_t mx = 4;
  for (auto v : P.ld) mx = std::max(mx, v);
  return mx;
}

size_t center_partial_bytes(const DevFactor& F, int64_t nrhs, size_t es) {
  if (F.n_center <= 0) return 0;
  const int64_t ch = center_chunk_rows(F.nx);
  const size_t nchunk = (size_t)((F.nx + ch - 1) / ch);
  return nchunk * (size_t)F.n_center * (size_t)nrhs * es;
}

// Workspace of the parts one after the other: two state buffers of the
// widest state, which the center's partial sums reuse.
size_t workspace_bytes_seq(const DevFactor& F, int prec, int64_t nrhs) {
  const size_t es = prec == MBF_C128 ? 16 : 8;
  return align256(std::max(2 * (size_t)state_ld_max(F) * (size_t)nrhs * es, center_partial_bytes(F, nrhs, es)));
}

// Workspace of the parts side by side: two state buffers per part, then the
// center's partial sums.  Offsets of the regions in `off` (parts, center).
size_t workspace_bytes_par(const DevFactor& F, int prec, int64_t nrhs, std::vector<size_t>* off) {
  const size_t es = prec == MBF_C128 ? 16 : 8;
  size_t b = 0;
  for (const auto& P : F.parts) {
    if (off) off->push_back(b);
    b += align256(2 * (size_t)part_ld_max(P) * (size_t)nrhs * es);
  }
  if (off) off->push_back(b);
  return b + align256(center_partial_bytes(F, nrhs, es));
}
}  // namespace

size_t workspace_bytes(const DevFactor& F, int prec, int64_t nrhs) {
  const size_t seq = workspace_bytes_seq(F, prec, nrhs);
  return F.parts.size() > 1 ? std::max(seq, workspace_bytes_par(F, prec, nrhs, nullptr)) : seq;
}

// ------------------------------------------------------------------ scratch
// Fixed device scratch of mbf_apply_scratch: the apply's workspace (the two
// stage-state buffers, and the dense center's partial sums of a multiscale
// adjoint) taken from a file-scope device array instead of caller memory.
// Each device that runs the library holds its own copy until the process
// ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.  No part of it needs
// to start at zero: every stage writes its whole output state before the
// next one reads it.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

Error scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return {MBF_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)};
  if (dev < 0 || dev >= kMaxDevices) return {MBF_ERR_UNSUPPORTED, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return {MBF_ERR_HIP, std::string("hipGetSymbolAddress (scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return {MBF_OK, ""};
}
}  // namespace

size_t scratch_bytes() { return kScratchBytes; }

Error launch_apply_scratch(const DevFactor& F, int prec, int64_t nrhs, const void* in, int64_t ldin, void* out,
                           int64_t ldout, hipStream_t st) {
  const size_t need = workspace_bytes_seq(F, prec, nrhs);  // the parts run one after the other here
  if (need > kScratchBytes)
    return {MBF_ERR_INVALID_ARG, "apply needs " + std::to_string(need) + " bytes of workspace, above the " +
                                     std::to_string(kScratchBytes) + "-byte device scratch: use mbf_apply"};
  void* ws = nullptr;
  Error e = scratch_address(&ws);
  if (e.st != MBF_OK) return e;
  return launch_apply(F, prec, false, nrhs, in, ldin, out, ldout, ws, kScratchBytes, st);
}

namespace {
// Side streams of one caller stream (per device) for the parts of a
// multiscale apply: the coronas' butterflies and the dense center of
// eq. (f1) are independent until their sums meet in u, so they run side by
// side.  Created on first use (default priority, non-blocking) and kept for
// the life of the process; `fork` orders them after the caller's earlier
// work, `done[i]` marks the end of side stream i's share.
struct SideStreams {
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
};
std::mutex g_side_mu;
std::map<std::pair<int, hipStream_t>, SideStreams> g_side;

Error side_streams(hipStream_t caller, size_t n, SideStreams** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return {MBF_ERR_HIP, "hipGetDevice"};
  std::lock_guard<std::mutex> g(g_side_mu);
  SideStreams& S = g_side[{dev, caller}];
  if (!S.fork && hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) != hipSuccess) {
    S.fork = nullptr;
    return {MBF_ERR_HIP, "hipEventCreateWithFlags"};
  }
  while (S.st.size() < n) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return {MBF_ERR_HIP, "hipStreamCreate"};
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      return {MBF_ERR_HIP, "hipEventCreateWithFlags"};
    }
    S.st.push_back(s);
    S.done.push_back(e);
  }
  *out = &S;
  return {MBF_OK, ""};
}

}  // namespace

void release_side_streams(hipStream_t caller) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> g(g_side_mu);
  auto it = g_side.find({dev, caller});
  if (it == g_side.end()) return;
  for (size_t i = 0; i < it->second.st.size(); ++i) {
    (void)hipStreamSynchronize(it->second.st[i]);
    (void)hipStreamDestroy(it->second.st[i]);
    (void)hipEventDestroy(it->second.done[i]);
  }
  if (it->second.fork) (void)hipEventDestroy(it->second.fork);
  g_side.erase(it);
}

namespace {
// MBF_PART_STREAMS=0 runs the parts of a multiscale apply one after the other.
bool parts_side_by_side() {
  const char* e = std::getenv("MBF_PART_STREAMS");
  return !(e && e[0] == '0');
}

// The multiscale apply with its parts side by side (see SideStreams).
// Forward: the center writes u first, then every part adds its sum in part
// order (each reconstruction waits for the previous one), the same order as
// one after the other, so the results are identical.  Adjoint: the parts
// and the center write disjoint entries of v and need no order.
template <typename T>
Error apply_side_by_side(const DevFactor& F, int prec, bool adj, int64_t nrhs, const void* in, int64_t ldin,
                         void* out, int64_t ldout, void* ws, hipStream_t st) {
  const size_t np = F.parts.size();
  const bool center = F.n_center > 0;
  const size_t nside = np + (center ? 1 : 0);
  SideStreams* S = nullptr;
  Error e = side_streams(st, nside, &S);
  if (e.st != MBF_OK) return e;
  std::vector<size_t> off;
  (void)workspace_bytes_par(F, prec, nrhs, &off);
  char* base = reinterpret_cast<char*>(ws);
  if (hipEventRecord(S->fork, st) != hipSuccess) return {MBF_ERR_HIP, "hipEventRecord"};
  size_t forked = 0;
  for (; forked < nside; ++forked)
    if (hipStreamWaitEvent(S->st[forked], S->fork, 0) != hipSuccess) break;
  if (forked < nside) e = {MBF_ERR_HIP, "hipStreamWaitEvent"};
  const int64_t ws_ld = state_ld_max(F);
  hipEvent_t prev = nullptr;  // forward: the last writer of u so far
  if (e.st == MBF_OK && center) {
    hipStream_t cs = S->st[np];
    e = run_center<T>(F, prec, adj, nrhs, in, ldin, out, ldout, base + off[np], false, cs);
    if (e.st == MBF_OK && hipEventRecord(S->done[np], cs) != hipSuccess) e = {MBF_ERR_HIP, "hipEventRecord"};
    prev = S->done[np];
  }
  for (size_t i = 0; i < np && e.st == MBF_OK; ++i) {
    const auto& P = F.parts[i];
    const bool acc = !adj && (center || i > 0);
    e = run_part<T>(P, (int)i, &F.prof, prec, adj, nrhs, in, ldin, out, ldout, base + off[i], ws_ld,
                    part_ld_max(P), acc, S->st[i], adj ? nullptr : prev, adj ? nullptr : S->done[i]);
    prev = S->done[i];
  }
  // join every side stream that was forked, also after an error, so that no
  // work of this call is left running behind the caller's stream
  for (size_t i = 0; i < forked; ++i)
    if (hipEventRecord(S->done[i], S->st[i]) != hipSuccess || hipStreamWaitEvent(st, S->done[i], 0) != hipSuccess)
      if (e.st == MBF_OK) e = {MBF_ERR_HIP, "join of the side streams"};
  return e;
}
}  // namespace

Error launch_apply(const DevFactor& F, int prec, bool adj, int64_t nrhs, const void* in, int64_t ldin,
                   void* out, int64_t ldout, void* ws, size_t ws_bytes, hipStream_t st) {
  if (nrhs <= 0) return {MBF_OK, ""};
  if (ws_bytes < workspace_bytes_seq(F, prec, nrhs)) return {MBF_ERR_INVALID_ARG, "workspace too small"};
  if (F.parts.size() > 1 && parts_side_by_side() && ws_bytes >= workspace_bytes_par(F, prec, nrhs, nullptr)) {
    // not while the caller's stream is being captured into a graph: the
    // side streams would have to join the capture
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      Error e = prec == MBF_C128 ? apply_side_by_side<double>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, st)
                                 : apply_side_by_side<float>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, st);
      if (e.st != MBF_OK) return e;
      return hip_check("apply launch");
    }
  }
  const int64_t ws_ld = state_ld_max(F);
  bool acc = false;
  if (F.n_center > 0 && !adj) {
    Error e = prec == MBF_C128 ? run_center<double>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, false, st)
                               : run_center<float>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, false, st);
    if (e.st != MBF_OK) return e;
    acc = true;
  }
  for (size_t i = 0; i < F.parts.size(); ++i) {
    const auto& P = F.parts[i];
    Error e = prec == MBF_C128 ? run_part<double>(P, (int)i, &F.prof, prec, adj, nrhs, in, ldin, out, ldout, ws,
                                                  ws_ld, ws_ld, acc && !adj, st)
                               : run_part<float>(P, (int)i, &F.prof, prec, adj, nrhs, in, ldin, out, ldout, ws,
                                                 ws_ld, ws_ld, acc && !adj, st);
    if (e.st != MBF_OK) return e;
    acc = true;
  }
  if (F.n_center > 0 && adj) {
    Error e = prec == MBF_C128 ? run_center<double>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, false, st)
                               : run_center<float>(F, prec, adj, nrhs, in, ldin, out, ldout, ws, false, st);
    if (e.st != MBF_OK) return e;
  }
  return {MBF_OK, ""};
}

}  // namespace mbf
