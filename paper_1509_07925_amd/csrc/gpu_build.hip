// FP64 builder on the GPU: the butterfly factorization of Section 2 from
// kernel entries (case (ii)), with every dense step on the device.
//
// Steps, in the paper's order:
//   * Middle level (Section 2.3, eq. (Kij)): for every pair (A at X-level h,
//     B at Omega-level L-h), the SVD of K_{A,B} via random sampling
//     (Section 2.1): representative columns by a pivoted QR of randomly
//     selected rows, representative rows by a pivoted QR of the
//     representative columns, orthonormal bases Q_col / Q_row of the
//     representative columns / rows, the middle matrix
//     M = pinv(Q_col(I_row,:)) K(I_row, I_col) pinv(Q_row(I_col,:)^*) on
//     index sets that contain the representatives, and the SVD of M; kept in
//     form 1 (eq. (lowrank1)).
//   * Recursive factorizations of U^h and V^h (Section 2.4, eq. (blockF),
//     eq. (RSh2)): level by level, the truncated SVD of every merged block
//     [U_{A, child_s B'} restricted to A_t]_s (and its mirror for V) in form 2
//     (eq. (lowrank2)).
//
// Device design.  All matrices are FP64 complex, column-major, batched with
// zero padding to the largest member of a batch.  Orthonormal bases,
// pseudo-inverses and truncated SVDs come from Gram matrices (rocBLAS
// ZHERK / ZGEMM) and batched Hermitian eigendecompositions (rocSOLVER
// ZHEEVD); the kernel entries, the pivoted QR of the sampled blocks, the
// merges, the rank selection and the conversion into the apply layout are
// kernels of this file.  The middle level keeps, per pair, the
// representative indices and two small coefficient matrices:
//     U_{A,B} = K(A, J) X_u,     V_{B,A} = K(I, B)^* X_v,
// so U^h and V^h (O(N^{3/2}) entries) are regenerated from kernel entries
// when the recursions need them instead of being stored.  The recursions'
// blocks are converted to every requested precision as each batch
// finishes, and the pieces of a stage are joined into one allocation at the
// end.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "gpu_build.h"

namespace mbf {
namespace {

using z2 = double2;

struct DevErr : std::runtime_error {
  mbf_status st;
  DevErr(mbf_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

void hipck(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw DevErr(e == hipErrorOutOfMemory ? MBF_ERR_OOM : MBF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
void rbck(rocblas_status e, const char* what) {
  if (e != rocblas_status_success)
    throw DevErr(e == rocblas_status_memory_error ? MBF_ERR_OOM : MBF_ERR_HIP,
                 std::string(what) + ": rocBLAS / rocSOLVER status " + std::to_string((int)e));
}

// Owned device allocation.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  explicit DBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    hipck(hipMalloc(&p, b), "hipMalloc (device builder)");
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DBuf() { release(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
  void* take() {
    void* q = p;
    p = nullptr;
    bytes = 0;
    return q;
  }
};

inline size_t zb(int64_t n) { return (size_t)std::max<int64_t>(n, 1) * sizeof(z2); }

// ------------------------------------------------------------------ entries
// Integer coordinates of the points and, for the FIO, c1 / c2 of every X
// point (Section 3.3, eq. (example1phi)).
struct KSpec {
  int kind;  // 0 = DFT, 1 = FIO
  int64_t n;
  const int32_t* xn1;
  const int32_t* xn2;
  const double* c1;
  const double* c2;
  const int32_t* w1;
  const int32_t* w2;
};

// K(x, xi): DFT exp(-2 pi i x.xi / n) with x.xi reduced modulo n exactly;
// FIO exp(2 pi i Phi), Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2), the
// integer part of n x.xi reduced modulo n before the division.
__device__ __forceinline__ z2 kentry(const KSpec& k, int32_t xr, int32_t oc) {
  const int64_t a1 = k.w1[oc], a2 = k.w2[oc];
  int64_t q = ((int64_t)k.xn1[xr] * a1 + (int64_t)k.xn2[xr] * a2) % k.n;
  if (q < 0) q += k.n;
  double s, c;
  if (k.kind == 0) {
    sincospi(-2.0 * ((double)q / (double)k.n), &s, &c);
  } else {
    const double c1 = k.c1[xr], c2 = k.c2[xr];
    const double w1 = (double)a1, w2 = (double)a2;
    double ph = (double)q / (double)k.n + sqrt(c1 * c1 * w1 * w1 + c2 * c2 * w2 * w2);
    ph -= floor(ph);
    sincospi(2.0 * ph, &s, &c);
  }
  return make_double2(c, s);
}

// One sampled block per batch member: rows index X (caller indices), cols
// index Omega; entries beyond nr / nc are zero.
struct EntryDesc {
  const int32_t* rows;
  const int32_t* cols;
  int32_t nr, nc;
};

// out[b * ostride + i * rs + j * cs] = K(rows[i], cols[j]) (conjugated when
// conj), i < NR, j < NC.  i_fast: consecutive threads walk i (rs == 1).
__global__ __launch_bounds__(256) void k_entries(KSpec ks, const EntryDesc* __restrict__ ed, int NR, int NC,
                                                 z2* __restrict__ out, int64_t ostride, int64_t rs, int64_t cs,
                                                 int conj, int i_fast) {
  const EntryDesc d = ed[blockIdx.y];
  z2* o = out + (int64_t)blockIdx.y * ostride;
  const int64_t total = (int64_t)NR * NC;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int i, j;
    if (i_fast) {
      i = (int)(e % NR);
      j = (int)(e / NR);
    } else {
      j = (int)(e % NC);
      i = (int)(e / NC);
    }
    z2 v = make_double2(0.0, 0.0);
    if (i < d.nr && j < d.nc) {
      v = kentry(ks, d.rows[i], d.cols[j]);
      if (conj) v.y = -v.y;
    }
    o[(int64_t)i * rs + (int64_t)j * cs] = v;
  }
}

// --------------------------------------------------------------- pivoted QR
// Column selection by Householder QR with column pivoting (Section 2.1:
// representative columns of sampled rows).  Z: row-major p x c per batch
// member (ldz >= c), rows [0, nrow_b) and columns [0, ncol_b) valid;
// overwritten.  One workgroup per member; thread t owns columns t + 256 k.
// Records pivots until the largest remaining column norm is at most rtol
// times the first pivot's, or kmax of them.
constexpr int kQrRows = 2048;
constexpr int kQrCols = 256 * 32;

template <int CPT>
__global__ __launch_bounds__(256) void k_qrcp(z2* __restrict__ Z, int64_t zstride, int ldz,
                                              const int32_t* __restrict__ nrow_b, const int32_t* __restrict__ ncol_b,
                                              int kmax, double rtol2, int32_t* __restrict__ piv,
                                              int32_t* __restrict__ kout) {
  __shared__ z2 v[kQrRows];
  __shared__ double red_v[4];
  __shared__ int red_i[4];
  __shared__ double sh_beta;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  z2* A = Z + (int64_t)b * zstride;
  const int nr = min(nrow_b[b], kQrRows), nc = ncol_b[b];
  double cn[CPT], cn0[CPT];
  unsigned act = 0;
#pragma unroll
  for (int t = 0; t < CPT; ++t) {
    const int j = tid + 256 * t;
    double s = 0.0;
    if (j < nc) {
      for (int i = 0; i < nr; ++i) {
        const z2 a = A[(int64_t)i * ldz + j];
        s += a.x * a.x + a.y * a.y;
      }
      act |= 1u << t;
    }
    cn[t] = cn0[t] = s;
  }
  double first = -1.0;
  int k = 0;
  const int kend = min(kmax, min(nr, nc));
  for (; k < kend; ++k) {
    double best = -1.0;
    int bj = -1;
#pragma unroll
    for (int t = 0; t < CPT; ++t)
      if (((act >> t) & 1u) && cn[t] > best) {
        best = cn[t];
        bj = tid + 256 * t;
      }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oj = __shfl_xor(bj, off);
      if (ob > best || (ob == best && oj >= 0 && (bj < 0 || oj < bj))) {
        best = ob;
        bj = oj;
      }
    }
    if (lane == 0) {
      red_v[wid] = best;
      red_i[wid] = bj;
    }
    __syncthreads();
    if (tid == 0) {
      double bb = red_v[0];
      int jj = red_i[0];
      for (int w = 1; w < 4; ++w)
        if (red_v[w] > bb || (red_v[w] == bb && red_i[w] >= 0 && (jj < 0 || red_i[w] < jj))) {
          bb = red_v[w];
          jj = red_i[w];
        }
      red_v[0] = bb;
      red_i[0] = jj;
    }
    __syncthreads();
    const double bmax = red_v[0];
    const int pc = red_i[0];
    if (k == 0) first = bmax;
    if (pc < 0 || !(bmax > 0.0) || bmax <= rtol2 * first) break;
    if ((pc & 255) == tid) act &= ~(1u << (pc >> 8));
    for (int i = k + tid; i < nr; i += 256) v[i] = A[(int64_t)i * ldz + pc];
    __syncthreads();
    if (wid == 0) {
      double s = 0.0;
      for (int i = k + lane; i < nr; i += 64) s += v[i].x * v[i].x + v[i].y * v[i].y;
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) {
        // H = I - beta v v^*, v = x + phase(x_k) |x| e_k, beta = 1 / (|x| (|x| + |x_k|))
        const double nrm = sqrt(s);
        const z2 x0 = v[k];
        const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
        const double pr = ax0 > 0.0 ? x0.x / ax0 : 1.0, pi = ax0 > 0.0 ? x0.y / ax0 : 0.0;
        v[k] = make_double2(x0.x + pr * nrm, x0.y + pi * nrm);
        sh_beta = nrm > 0.0 ? 1.0 / (nrm * (nrm + ax0)) : 0.0;
        piv[(int64_t)b * kmax + k] = pc;
      }
    }
    __syncthreads();
    const double beta = sh_beta;
    z2 w[CPT];
#pragma unroll
    for (int t = 0; t < CPT; ++t) w[t] = make_double2(0.0, 0.0);
    for (int i = k; i < nr; ++i) {
      const z2 vi = v[i];
      const z2* row = A + (int64_t)i * ldz;
#pragma unroll
      for (int t = 0; t < CPT; ++t)
        if ((act >> t) & 1u) {
          const z2 a = row[tid + 256 * t];
          w[t].x += vi.x * a.x + vi.y * a.y;
          w[t].y += vi.x * a.y - vi.y * a.x;
        }
    }
    for (int i = k; i < nr; ++i) {
      const z2 vi = v[i];
      z2* row = A + (int64_t)i * ldz;
#pragma unroll
      for (int t = 0; t < CPT; ++t)
        if ((act >> t) & 1u) {
          z2 a = row[tid + 256 * t];
          a.x -= beta * (vi.x * w[t].x - vi.y * w[t].y);
          a.y -= beta * (vi.x * w[t].y + vi.y * w[t].x);
          row[tid + 256 * t] = a;
          if (i == k) cn[t] -= a.x * a.x + a.y * a.y;
        }
    }
#pragma unroll
    for (int t = 0; t < CPT; ++t)
      if (((act >> t) & 1u) && cn[t] <= 1e-8 * cn0[t]) {
        const int j = tid + 256 * t;
        double s = 0.0;
        for (int i = k + 1; i < nr; ++i) {
          const z2 a = A[(int64_t)i * ldz + j];
          s += a.x * a.x + a.y * a.y;
        }
        cn[t] = cn0[t] = s;
      }
    __syncthreads();
  }
  if (tid == 0) kout[b] = k;
}

// ------------------------------------------------------- eigen selections
// After ZHEEVD (eigenvectors in the columns of V, d x d with ld d, and
// eigenvalues ascending): count[b] = number of largest eigenvalues lam with
// lam > thr * lam_max and lam > 0, at most cap.
__global__ void k_eig_count(const double* __restrict__ D, int d, int64_t dstride, double thr, int cap,
                            int32_t* __restrict__ count, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double* lam = D + (int64_t)b * dstride;
  const double lmax = d > 0 ? lam[d - 1] : 0.0;
  int c = 0;
  if (lmax > 0.0)
    while (c < d && c < cap && lam[d - 1 - c] > thr * lmax) ++c;
  count[b] = c;
}

// o1[:, j] = V[:, d-1-j] * f1(lam), o2 likewise with f2, for j < count[b];
// zero columns for count[b] <= j < ncol.  f: 0 -> 1, 1 -> 1/sqrt(lam),
// 2 -> sqrt(lam).  sig[j] = sqrt(lam) (0 beyond the count).
__global__ __launch_bounds__(256) void k_eig_take(const z2* __restrict__ V, int d, int64_t vstride,
                                                  const double* __restrict__ D, int64_t dstride,
                                                  const int32_t* __restrict__ count, int ncol, int f1,
                                                  z2* __restrict__ o1, int64_t o1stride, int ld1, int f2,
                                                  z2* __restrict__ o2, int64_t o2stride, int ld2,
                                                  double* __restrict__ sig, int64_t sstride) {
  const int b = blockIdx.y;
  const double* lam = D + (int64_t)b * dstride;
  const int cnt = count[b];
  const z2* Vb = V + (int64_t)b * vstride;
  const int64_t total = (int64_t)d * ncol;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % d), j = (int)(e / d);
    z2 x1 = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
    if (j < cnt) {
      const double l = lam[d - 1 - j];
      const z2 vv = Vb[(int64_t)(d - 1 - j) * d + i];
      const double s1 = f1 == 0 ? 1.0 : (f1 == 1 ? 1.0 / sqrt(l) : sqrt(l));
      const double s2 = f2 == 0 ? 1.0 : (f2 == 1 ? 1.0 / sqrt(l) : sqrt(l));
      x1 = make_double2(vv.x * s1, vv.y * s1);
      x2 = make_double2(vv.x * s2, vv.y * s2);
    }
    if (o1) o1[(int64_t)b * o1stride + i + (int64_t)j * ld1] = x1;
    if (o2) o2[(int64_t)b * o2stride + i + (int64_t)j * ld2] = x2;
  }
  if (sig && blockIdx.x == 0)
    for (int j = threadIdx.x; j < ncol; j += 256) sig[(int64_t)b * sstride + j] = j < cnt ? sqrt(lam[d - 1 - j]) : 0.0;
}

// ------------------------------------------------------------------ merges
// W (P x Kmax per member) = [S_0(rows) S_1(rows) S_2(rows) S_3(rows)]: the
// columns of up to four source matrices (nc[s] columns each, leading
// dimension ld[s]) restricted to rows [row0, row0 + nrow), zero padded.
struct GatherDesc {
  const z2* src[4];
  int32_t ld[4];
  int32_t nc[4];
  int32_t row0, nrow;
};

__global__ __launch_bounds__(256) void k_gather(const GatherDesc* __restrict__ gd, int P, int Kmax,
                                                z2* __restrict__ W, int64_t wstride) {
  const GatherDesc d = gd[blockIdx.y];
  z2* o = W + (int64_t)blockIdx.y * wstride;
  const int c1 = d.nc[0], c2 = c1 + d.nc[1], c3 = c2 + d.nc[2], c4 = c3 + d.nc[3];
  const int64_t total = (int64_t)P * Kmax;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % P), j = (int)(e / P);
    z2 v = make_double2(0.0, 0.0);
    if (i < d.nrow && j < c4) {
      const bool s0 = j < c1, s1 = j < c2, s2 = j < c3;
      const z2* sp = s0 ? d.src[0] : (s1 ? d.src[1] : (s2 ? d.src[2] : d.src[3]));
      const int ld = s0 ? d.ld[0] : (s1 ? d.ld[1] : (s2 ? d.ld[2] : d.ld[3]));
      const int jj = j - (s0 ? 0 : (s1 ? c1 : (s2 ? c2 : c3)));
      v = sp[(int64_t)d.row0 + i + (int64_t)jj * ld];
    }
    o[e] = v;
  }
}

// dst[b] (NR x K) = rows idx[b][i] of src[b] (zero for idx < 0).
__global__ __launch_bounds__(256) void k_gather_rows(const z2* __restrict__ src, int64_t sstride, int lds,
                                                     const int32_t* __restrict__ idx, int64_t istride, int NR, int K,
                                                     z2* __restrict__ dst, int64_t dstride) {
  const int b = blockIdx.y;
  const int64_t total = (int64_t)NR * K;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % NR), k = (int)(e / NR);
    const int32_t id = idx[(int64_t)b * istride + i];
    dst[(int64_t)b * dstride + e] = id >= 0 ? src[(int64_t)b * sstride + id + (int64_t)k * lds] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------- apply layout
// One factor piece into a stage block (column-major, M rows):
//   dst[(c0 + j) * M + r0 + i] = value(i, j),  i < ni, j < nj,
//   value(i, j) = src[i + j ld]            (tconj = 0)
//               = conj(src[j + i ld])      (tconj = 1)
// written in each requested precision: complex128, complex64, and the
// split BF16 form (re_hi, im_hi, re_lo, im_lo; hi = bf16(x), lo = bf16(x - hi),
// both rounded to nearest even).
struct PackDesc {
  const z2* src;
  int64_t dst;
  int32_t ld, ni, nj, M, r0, c0, tconj, pad;
};

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_pack(const PackDesc* __restrict__ pd, z2* __restrict__ o128,
                                              float2* __restrict__ o64, ushort4* __restrict__ obf) {
  const PackDesc d = pd[blockIdx.y];
  const int64_t total = (int64_t)d.ni * d.nj;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % d.ni), j = (int)(e / d.ni);
    z2 v;
    if (d.tconj) {
      v = d.src[j + (int64_t)i * d.ld];
      v.y = -v.y;
    } else {
      v = d.src[i + (int64_t)j * d.ld];
    }
    const int64_t o = d.dst + (int64_t)(d.c0 + j) * d.M + d.r0 + i;
    if (o128) o128[o] = v;
    const float re = (float)v.x, im = (float)v.y;
    if (o64) o64[o] = make_float2(re, im);
    if (obf) {
      const uint16_t rh = bf16_rne(re), ih = bf16_rne(im);
      const float rhf = __uint_as_float((uint32_t)rh << 16), ihf = __uint_as_float((uint32_t)ih << 16);
      obf[o] = make_ushort4(rh, ih, bf16_rne(re - rhf), bf16_rne(im - ihf));
    }
  }
}

// Leaf factor |leaf| x r (column-major at dst) from a level matrix.
struct LeafPack {
  const z2* src;
  int64_t dst;
  int32_t ld, np, r, pad;
};

__global__ __launch_bounds__(256) void k_pack_leaf(const LeafPack* __restrict__ lp, z2* __restrict__ o128,
                                                   float2* __restrict__ o64) {
  const LeafPack d = lp[blockIdx.y];
  const int64_t total = (int64_t)d.np * d.r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % d.np), k = (int)(e / d.np);
    const z2 v = d.src[i + (int64_t)k * d.ld];
    if (o128) o128[d.dst + e] = v;
    if (o64) o64[d.dst + e] = make_float2((float)v.x, (float)v.y);
  }
}

// Middle scaling S = Sigma^{-1} (eq. (lowrank1)) in state order.
__global__ void k_pack_s(const double* __restrict__ sig, int64_t sstride, const int32_t* __restrict__ r,
                         const int64_t* __restrict__ roff, int np, double* __restrict__ o128,
                         float* __restrict__ o32) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  for (int k = 0; k < r[p]; ++k) {
    const double v = 1.0 / sig[(int64_t)p * sstride + k];
    if (o128) o128[roff[p] + k] = v;
    if (o32) o32[roff[p] + k] = (float)v;
  }
}

// ZHERK writes the upper triangle only: mirror it into the lower triangle
// (conjugated) and make the diagonal real, so every Gram matrix handed to
// the eigensolvers is a complete Hermitian matrix.
__global__ void k_mirror_upper(z2* __restrict__ G, int n, int64_t sA, int batch) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n * batch) return;
  const int b = (int)(e / ((int64_t)n * n));
  const int64_t r = e % ((int64_t)n * n);
  const int i = (int)(r % n), j = (int)(r / n);
  z2* g = G + (int64_t)b * sA;
  if (i > j) {
    const z2 u = g[(int64_t)i * n + j];
    g[(int64_t)j * n + i] = make_double2(u.x, -u.y);
  } else if (i == j) {
    g[(int64_t)j * n + i].y = 0.0;
  }
}

// Valid size of a zero-padded Hermitian matrix: 1 + the last row with a
// nonzero entry (0 for the zero matrix).  Padding always trails.
__global__ void k_valid_size(const z2* __restrict__ G, int n, int64_t sA, int batch, int32_t* __restrict__ v) {
  const int b = blockIdx.x;
  if (b >= batch) return;
  const z2* g = G + (int64_t)b * sA;
  __shared__ int last;
  if (threadIdx.x == 0) last = -1;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const z2 x = g[e];
    if (x.x != 0.0 || x.y != 0.0) atomicMax(&last, (int)(e % n));
  }
  __syncthreads();
  if (threadIdx.x == 0) v[b] = last + 1;
}

// Leading v x v blocks of the listed members into a dense v x v batch.
__global__ void k_take_block(const z2* __restrict__ G, int n, int64_t sA, const int32_t* __restrict__ members, int v,
                             z2* __restrict__ out) {
  const int k = blockIdx.y;
  const z2* g = G + (int64_t)members[k] * sA;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)v * v; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % v), j = (int)(e / v);
    out[(int64_t)k * v * v + e] = g[(int64_t)j * n + i];
  }
}

// Eigenpairs of the v x v blocks back into the n x n layout: the v pairs in
// the top positions (ascending), padded coordinates zero; the n - v padded
// directions get eigenvalue -1 and zero vectors (never selected).
__global__ void k_put_eig(z2* __restrict__ G, int n, int64_t sA, double* __restrict__ D, const int32_t* __restrict__ members,
                          int v, const z2* __restrict__ vec, const double* __restrict__ val) {
  const int k = blockIdx.y;
  const int b = members[k];
  z2* g = G + (int64_t)b * sA;
  const int off = n - v;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)n * n; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % n), j = (int)(e / n);
    z2 x = make_double2(0.0, 0.0);
    if (j >= off && i < v) x = vec[(int64_t)k * v * v + (int64_t)(j - off) * v + i];
    g[e] = x;
  }
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < n; j += blockDim.x) D[(int64_t)b * n + j] = j >= off ? val[(int64_t)k * v + (j - off)] : -1.0;
}

// 1 for members whose eigenpairs are not all finite.
__global__ void k_nonfinite(const z2* __restrict__ V, const double* __restrict__ D, int v, int batch,
                            int32_t* __restrict__ flag) {
  const int b = blockIdx.x;
  if (b >= batch) return;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)v * v; e += blockDim.x) {
    const z2 x = V[(int64_t)b * v * v + e];
    if (!isfinite(x.x) || !isfinite(x.y)) bad = 1;
  }
  for (int j = threadIdx.x; j < v; j += blockDim.x)
    if (!isfinite(D[(int64_t)b * v + j])) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) flag[b] = bad;
}

// ------------------------------------------------------------- launchers
inline unsigned gridx(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 2048));
}

bool verbose() { return std::getenv("MBF_VERBOSE") != nullptr; }

// Wall time per kind of work, gathered only with MBF_VERBOSE (each mark
// waits for the stream).
enum TimeCat { T_ENTRIES, T_QRCP, T_BLAS, T_EIG, T_EIG_REDO, T_SMALL, T_HOST, T_NCAT };
const char* kCatName[T_NCAT] = {"entries", "pivoted QR", "GEMM/HERK", "eigensolver", "eigensolver redo",
                                "small kernels", "host"};
struct Timers {
  double acc[T_NCAT] = {0};
  std::chrono::steady_clock::time_point last = std::chrono::steady_clock::now();
  void mark(hipStream_t st, TimeCat c) {
    if (!verbose()) return;
    (void)hipStreamSynchronize(st);
    const auto now = std::chrono::steady_clock::now();
    acc[c] += std::chrono::duration<double>(now - last).count();
    last = now;
  }
  void report(const char* what) {
    if (!verbose()) return;
    std::fprintf(stderr, "[mbf device build] time by kind after %s:", what);
    for (int c = 0; c < T_NCAT; ++c) std::fprintf(stderr, " %s %.2fs;", kCatName[c], acc[c]);
    std::fprintf(stderr, "\n");
    std::fflush(stderr);
  }
};
Timers g_tm;

struct DBufLite {
  void* p = nullptr;
  size_t bytes = 0;
  explicit DBufLite(size_t b) : bytes(b) { hipck(hipMalloc(&p, std::max<size_t>(b, 1)), "hipMalloc (eigensolver)"); }
  ~DBufLite() { (void)hipFree(p); }
  DBufLite(const DBufLite&) = delete;
  DBufLite& operator=(const DBufLite&) = delete;
};

struct Blas {
  rocblas_handle h = nullptr;
  hipStream_t st = nullptr;
  ~Blas() {
    if (h) (void)rocblas_destroy_handle(h);
  }
  void gemm(rocblas_operation ta, rocblas_operation tb, int m, int n, int k, const z2* A, int lda, int64_t sA,
            const z2* B, int ldb, int64_t sB, z2* C, int ldc, int64_t sC, int batch) {
    if (m <= 0 || n <= 0 || batch <= 0) return;
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    if (k <= 0) {
      // C = 0: a product with an empty inner dimension
      for (int b = 0; b < batch; ++b)
        hipck(hipMemset2DAsync(C + (int64_t)b * sC, (size_t)ldc * sizeof(z2), 0, (size_t)m * sizeof(z2), (size_t)n,
                               st),
              "hipMemset2DAsync");
      return;
    }
    rbck(rocblas_zgemm_strided_batched(h, ta, tb, m, n, k, &one, reinterpret_cast<const rocblas_double_complex*>(A),
                                       lda, sA, reinterpret_cast<const rocblas_double_complex*>(B), ldb, sB, &zero,
                                       reinterpret_cast<rocblas_double_complex*>(C), ldc, sC, batch),
         "zgemm");
    g_tm.mark(st, T_BLAS);
  }
  // C (n x n, upper triangle) = A^* A (A is k x n) when ah, else A A^* (A is n x k)
  void herk(bool ah, int n, int k, const z2* A, int lda, int64_t sA, z2* C, int ldc, int64_t sC, int batch) {
    if (n <= 0 || batch <= 0) return;
    const double one = 1.0, zero = 0.0;
    rbck(rocblas_zherk_strided_batched(h, rocblas_fill_upper,
                                       ah ? rocblas_operation_conjugate_transpose : rocblas_operation_none, n,
                                       std::max(k, 0), &one, reinterpret_cast<const rocblas_double_complex*>(A),
                                       std::max(lda, 1), sA, &zero, reinterpret_cast<rocblas_double_complex*>(C), ldc,
                                       sC, batch),
         "zherk");
    g_tm.mark(st, T_BLAS);
  }
  // Eigendecomposition of Hermitian n x n matrices (upper triangle given),
  // in place: eigenvectors in the columns, eigenvalues ascending in D.
  // Members are zero-padded; the divide-and-conquer solver (ZHEEVD) returns
  // non-finite vectors on matrices with such decoupled zero rows, so every
  // member's leading nonzero block (its valid size v) is solved on its own,
  // grouped by v, and put back with the padded directions at eigenvalue -1.
  // Members whose divide-and-conquer result is not finite or did not converge
  // are solved again by QR iteration (ZHEEV).
  void heevd(int n, z2* A, int64_t sA, double* D, double* E, int32_t* info, int batch) {
    (void)E;
    (void)info;
    if (n <= 0 || batch <= 0) return;
    g_tm.mark(st, T_HOST);
    hipLaunchKernelGGL(k_mirror_upper, dim3((unsigned)(((int64_t)n * n * batch + 255) / 256)), dim3(256), 0, st, A, n,
                       sA, batch);
    hipck(hipGetLastError(), "k_mirror_upper");
    int32_t* dv = nullptr;
    hipck(hipMalloc(&dv, (size_t)batch * 4), "hipMalloc");
    struct Free {
      void* p;
      ~Free() { (void)hipFree(p); }
    } fv{dv};
    hipLaunchKernelGGL(k_valid_size, dim3(batch), dim3(256), 0, st, A, n, sA, batch, dv);
    hipck(hipGetLastError(), "k_valid_size");
    std::vector<int32_t> hv(batch);
    hipck(hipMemcpyAsync(hv.data(), dv, (size_t)batch * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<std::vector<int32_t>> groups(n + 1);
    for (int b = 0; b < batch; ++b) groups[hv[b]].push_back(b);
    for (int v = 0; v <= n; ++v) {
      const std::vector<int32_t>& mem = groups[v];
      if (mem.empty()) continue;
      const int nm = (int)mem.size();
      DBufLite dmem((size_t)nm * 4), blk((size_t)std::max(v, 1) * std::max(v, 1) * sizeof(z2) * nm),
          val((size_t)std::max(v, 1) * 8 * nm), off((size_t)std::max(v, 1) * 8 * nm), inf((size_t)nm * 4),
          flag((size_t)nm * 4);
      hipck(hipMemcpyAsync(dmem.p, mem.data(), (size_t)nm * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      if (v > 0) {
        hipLaunchKernelGGL(k_take_block, dim3(gridx((int64_t)v * v), nm), dim3(256), 0, st, A, n, sA,
                           (const int32_t*)dmem.p, v, (z2*)blk.p);
        hipck(hipGetLastError(), "k_take_block");
        // keep the inputs for a possible second solve
        DBufLite keep((size_t)v * v * sizeof(z2) * nm);
        hipck(hipMemcpyAsync(keep.p, blk.p, keep.bytes, hipMemcpyDeviceToDevice, st), "copy");
        rbck(rocsolver_zheevd_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, v,
                                              (rocblas_double_complex*)blk.p, v, (rocblas_stride)v * v, (double*)val.p, v,
                                              (double*)off.p, v, (rocblas_int*)inf.p, nm),
             "zheevd");
        g_tm.mark(st, T_EIG);
        hipLaunchKernelGGL(k_nonfinite, dim3(nm), dim3(256), 0, st, (const z2*)blk.p, (const double*)val.p, v, nm,
                           (int32_t*)flag.p);
        hipck(hipGetLastError(), "k_nonfinite");
        std::vector<int32_t> hi(nm), hf(nm);
        hipck(hipMemcpyAsync(hi.data(), inf.p, (size_t)nm * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hipck(hipMemcpyAsync(hf.data(), flag.p, (size_t)nm * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
        std::vector<int32_t> redo;
        for (int k = 0; k < nm; ++k)
          if (hi[k] != 0 || hf[k] != 0) redo.push_back(k);
        if (!redo.empty()) {
          const int nr = (int)redo.size();
          const size_t mb = (size_t)v * v * sizeof(z2);
          DBufLite rb(mb * nr), rv((size_t)v * 8 * nr), ro((size_t)v * 8 * nr), ri((size_t)nr * 4);
          for (int k = 0; k < nr; ++k)
            hipck(hipMemcpyAsync((char*)rb.p + mb * k, (char*)keep.p + mb * redo[k], mb, hipMemcpyDeviceToDevice, st),
                  "copy");
          rbck(rocsolver_zheev_strided_batched(h, rocblas_evect_original, rocblas_fill_upper, v,
                                               (rocblas_double_complex*)rb.p, v, (rocblas_stride)v * v, (double*)rv.p,
                                               v, (double*)ro.p, v, (rocblas_int*)ri.p, nr),
               "zheev");
          std::vector<int32_t> hr(nr);
          hipck(hipMemcpyAsync(hr.data(), ri.p, (size_t)nr * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
          hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
          for (int k = 0; k < nr; ++k) {
            if (hr[k] != 0)
              throw DevErr(MBF_ERR_HIP, "eigendecomposition did not converge (n = " + std::to_string(v) + ")");
            hipck(hipMemcpyAsync((char*)blk.p + mb * redo[k], (char*)rb.p + mb * k, mb, hipMemcpyDeviceToDevice, st),
                  "copy");
            hipck(hipMemcpyAsync((char*)val.p + (size_t)v * 8 * redo[k], (char*)rv.p + (size_t)v * 8 * k, (size_t)v * 8,
                                 hipMemcpyDeviceToDevice, st),
                  "copy");
          }
          g_tm.mark(st, T_EIG_REDO);
          if (std::getenv("MBF_VERBOSE_SOLVER"))
            std::fprintf(stderr, "[mbf device build] %d of %d eigendecompositions (n = %d) redone by QR iteration\n", nr,
                         nm, v);
        }
      }
      hipLaunchKernelGGL(k_put_eig, dim3(gridx((int64_t)n * n), nm), dim3(256), 0, st, A, n, sA, D,
                         (const int32_t*)dmem.p, v, (const z2*)blk.p, (const double*)val.p);
      hipck(hipGetLastError(), "k_put_eig");
      hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
      g_tm.mark(st, T_SMALL);
    }
  }
  static bool verbose_solver() { return std::getenv("MBF_VERBOSE") != nullptr; }
};

uint64_t mix(uint64_t a, uint64_t b) {
  uint64_t z = a * 0x9E3779B97F4A7C15ull + b + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// k distinct indices of [0, n), sorted.
std::vector<int32_t> sample(std::mt19937_64& rng, int32_t n, int32_t k) {
  k = std::min(k, n);
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  for (int32_t i = 0; i < k; ++i) {
    std::uniform_int_distribution<int32_t> d(i, n - 1);
    std::swap(all[i], all[d(rng)]);
  }
  all.resize(k);
  std::sort(all.begin(), all.end());
  return all;
}

std::vector<int32_t> merge_sorted(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  std::vector<int32_t> out;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}

template <typename T>
DBuf upload(const std::vector<T>& v, hipStream_t st) {
  DBuf d(std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) {
    hipck(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  return d;
}

template <typename T>
std::vector<T> download(const void* d, size_t n, hipStream_t st) {
  std::vector<T> v(n);
  if (n) {
    hipck(hipMemcpyAsync(v.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  return v;
}

// Matrices of one level, one per pair (A-major, B-minor): ptr / ld / rank;
// the storage is a list of batch buffers.
struct Mats {
  std::vector<DBuf> bufs;
  std::vector<const z2*> ptr;
  std::vector<int32_t> ld;
  void reset(size_t n) {
    bufs.clear();
    ptr.assign(n, nullptr);
    ld.assign(n, 1);
  }
};

// Blocks of one stage written so far, in block order: one piece per batch
// and precision.
struct Piece {
  void* p[kNumPrec] = {nullptr, nullptr, nullptr};
  int64_t elems = 0;
};



struct Builder {
  const Tree& xt;
  const Tree& ot;
  int L, m;
  const mbf_opts& o;
  uint32_t mask;
  double tol;
  int rmax, os;
  size_t budget;
  hipStream_t st = nullptr;
  Blas bl;
  KSpec ks{};
  DBuf d_xn1, d_xn2, d_c1, d_c2, d_w1, d_w2, d_xcall, d_ocall;
  std::vector<int32_t> xcall, ocall;
  std::vector<std::vector<int32_t>> rank;
  std::vector<std::vector<Piece>> pieces;  // [stage]
  Mats u_leaves, v_leaves;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  // Middle-level store (form 1 through regenerable factors): per pair,
  // J (caller indices, KCAP), X_u (KCAP x RCAP), I (caller indices, NICAP),
  // X_v (NICAP x RCAP), sigma (RCAP).
  int q = 0, KCAP = 0, NICAP = 0, RCAP = 0;
  DBuf mJ, mXu, mI, mXv, mSig;
  std::vector<int32_t> m_kc, m_ni;

  Builder(const Tree& x, const Tree& w, const mbf_opts& opts, uint32_t pm)
      : xt(x), ot(w), L(x.L), m(x.L / 2), o(opts), mask(pm), tol(opts.tol), rmax(opts.max_rank),
        os(opts.oversample) {
    if (opts.device_mem_gb > 0) {
      budget = (size_t)opts.device_mem_gb << 30;
    } else {
      // By default a third of the memory free when this part starts, between
      // 48 GiB and 128 GiB (less when less is free): bigger batches keep the
      // one-workgroup-per-pair kernels of the middle level busy, and what is
      // left holds the level matrices and the factors built so far.
      size_t fr = 0, tot = 0;
      const size_t gib = (size_t)1 << 30;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
      budget = std::min<size_t>(std::max<size_t>(48 * gib, fr / 3), 128 * gib);
      if (fr > 0) budget = std::min<size_t>(budget, fr / 10 * 9);
    }
  }
  ~Builder() {
    for (auto& v : pieces)
      for (auto& pc : v)
        for (void* p : pc.p)
          if (p) (void)hipFree(p);
    if (st) (void)hipStreamDestroy(st);
  }

  double secs() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  void log(const char* what) const {
    if (verbose()) {
      std::fprintf(stderr, "[mbf device build] %6.1fs %s\n", secs(), what);
      std::fflush(stderr);
    }
  }

  int64_t xsize(int l, int32_t i) const { return xt.size(l, i); }
  int64_t osize(int l, int32_t i) const { return ot.size(l, i); }
  int64_t pair(int s, int32_t ia, int32_t ib) const { return (int64_t)ia * ot.nn(L - s) + ib; }

  void entries(const std::vector<EntryDesc>& ed, int NR, int NC, z2* out, int64_t ostride, int64_t rs, int64_t cs,
               bool conj) {
    if (ed.empty() || NR <= 0 || NC <= 0) return;
    DBuf d = upload(ed, st);
    const bool i_fast = rs == 1;
    hipLaunchKernelGGL(k_entries, dim3(gridx((int64_t)NR * NC), (unsigned)ed.size()), dim3(256), 0, st, ks,
                       d.as<EntryDesc>(), NR, NC, out, ostride, rs, cs, conj ? 1 : 0, i_fast ? 1 : 0);
    hipck(hipGetLastError(), "k_entries");
    hipck(hipStreamSynchronize(st), "k_entries");
    g_tm.mark(st, T_ENTRIES);
  }

  // Pivoted QR selection on nb row-major p x c matrices.
  void qrcp(z2* Z, int64_t zstride, int ldz, const std::vector<int32_t>& nrow, const std::vector<int32_t>& ncol,
            int cmax, int kmax, double rtol, std::vector<int32_t>& piv, std::vector<int32_t>& kout) {
    const int nb = (int)nrow.size();
    for (int v : nrow)
      if (v > kQrRows) throw DevErr(MBF_ERR_UNSUPPORTED, "sampled block taller than the pivoted-QR kernel allows");
    DBuf dn = upload(nrow, st), dc = upload(ncol, st);
    DBuf dp((size_t)nb * std::max(kmax, 1) * 4), dk((size_t)nb * 4);
    hipck(hipMemsetAsync(dp.p, 0xff, dp.bytes, st), "hipMemsetAsync");
    const double r2 = rtol * rtol;
    g_tm.mark(st, T_HOST);
    if (cmax <= 256 * 4)
      hipLaunchKernelGGL(k_qrcp<4>, dim3(nb), dim3(256), 0, st, Z, zstride, ldz, dn.as<int32_t>(), dc.as<int32_t>(),
                         kmax, r2, dp.as<int32_t>(), dk.as<int32_t>());
    else if (cmax <= 256 * 8)
      hipLaunchKernelGGL(k_qrcp<8>, dim3(nb), dim3(256), 0, st, Z, zstride, ldz, dn.as<int32_t>(), dc.as<int32_t>(),
                         kmax, r2, dp.as<int32_t>(), dk.as<int32_t>());
    else if (cmax <= 256 * 16)
      hipLaunchKernelGGL(k_qrcp<16>, dim3(nb), dim3(256), 0, st, Z, zstride, ldz, dn.as<int32_t>(),
                         dc.as<int32_t>(), kmax, r2, dp.as<int32_t>(), dk.as<int32_t>());
    else if (cmax <= 256 * 32)
      hipLaunchKernelGGL(k_qrcp<32>, dim3(nb), dim3(256), 0, st, Z, zstride, ldz, dn.as<int32_t>(),
                         dc.as<int32_t>(), kmax, r2, dp.as<int32_t>(), dk.as<int32_t>());
    else
      throw DevErr(MBF_ERR_UNSUPPORTED, "sampled block wider than the pivoted-QR kernel allows");
    hipck(hipGetLastError(), "k_qrcp");
    piv = download<int32_t>(dp.p, (size_t)nb * kmax, st);
    kout = download<int32_t>(dk.p, (size_t)nb, st);
    g_tm.mark(st, T_QRCP);
  }

  // count of kept eigenvalues per member (device) and on the host
  std::vector<int32_t> eig_count(const double* D, int d, int nb, double thr, int cap, DBuf& dcnt) {
    dcnt.alloc((size_t)nb * 4);
    hipLaunchKernelGGL(k_eig_count, dim3((nb + 255) / 256), dim3(256), 0, st, D, d, (int64_t)d, thr, cap,
                       dcnt.as<int32_t>(), nb);
    hipck(hipGetLastError(), "k_eig_count");
    std::vector<int32_t> c = download<int32_t>(dcnt.p, (size_t)nb, st);
    g_tm.mark(st, T_SMALL);
    return c;
  }

  void eig_take(const z2* V, int d, const double* D, const int32_t* cnt, int nb, int ncol, int f1, z2* o1,
                int64_t s1, int ld1, int f2, z2* o2, int64_t s2, int ld2, double* sig, int64_t sst) {
    if (d <= 0 || ncol <= 0 || nb <= 0) return;
    hipLaunchKernelGGL(k_eig_take, dim3(gridx((int64_t)d * ncol), nb), dim3(256), 0, st, V, d, (int64_t)d * d, D,
                       (int64_t)d, cnt, ncol, f1, o1, s1, ld1, f2, o2, s2, ld2, sig, sst);
    hipck(hipGetLastError(), "k_eig_take");
    g_tm.mark(st, T_SMALL);
  }

  // Hermitian eigendecomposition of the Gram matrix of X (P x K, batch):
  // G = X^* X, eigenvectors in G, eigenvalues in D.
  void gram_eig(const z2* X, int P, int K, int nb, DBuf& G, DBuf& D) {
    G.alloc(zb((int64_t)nb * K * K));
    D.alloc((size_t)std::max(nb * K, 1) * 8);
    DBuf E((size_t)std::max(nb * K, 1) * 8), info((size_t)nb * 4);
    bl.herk(true, K, P, X, P, (int64_t)P * K, G.as<z2>(), K, (int64_t)K * K, nb);
    bl.heevd(K, G.as<z2>(), (int64_t)K * K, D.as<double>(), E.as<double>(), info.as<int32_t>(), nb);
  }

  // T (K x K) with Q = X T of orthonormal columns spanning the columns of X
  // above 1e-7 of its largest singular value: two passes of
  // T_k = V_k Lambda_k^{-1/2} from the Gram eigendecomposition.
  void orth(const z2* X, int P, int K, int nb, z2* Q, z2* T) {
    if (K <= 0) return;
    DBuf G, D, cnt, T1((zb((int64_t)nb * K * K))), Q1(zb((int64_t)nb * P * K)), T2(zb((int64_t)nb * K * K));
    gram_eig(X, P, K, nb, G, D);
    eig_count(D.as<double>(), K, nb, 1e-14, K, cnt);
    eig_take(G.as<z2>(), K, D.as<double>(), cnt.as<int32_t>(), nb, K, 1, T1.as<z2>(), (int64_t)K * K, K, 0, nullptr,
             0, 1, nullptr, 0);
    bl.gemm(rocblas_operation_none, rocblas_operation_none, P, K, K, X, P, (int64_t)P * K, T1.as<z2>(), K,
            (int64_t)K * K, Q1.as<z2>(), P, (int64_t)P * K, nb);
    gram_eig(Q1.as<z2>(), P, K, nb, G, D);
    eig_count(D.as<double>(), K, nb, 1e-14, K, cnt);
    eig_take(G.as<z2>(), K, D.as<double>(), cnt.as<int32_t>(), nb, K, 1, T2.as<z2>(), (int64_t)K * K, K, 0, nullptr,
             0, 1, nullptr, 0);
    bl.gemm(rocblas_operation_none, rocblas_operation_none, P, K, K, Q1.as<z2>(), P, (int64_t)P * K, T2.as<z2>(), K,
            (int64_t)K * K, Q, P, (int64_t)P * K, nb);
    bl.gemm(rocblas_operation_none, rocblas_operation_none, K, K, K, T1.as<z2>(), K, (int64_t)K * K, T2.as<z2>(), K,
            (int64_t)K * K, T, K, (int64_t)K * K, nb);
  }

  // Pseudo-inverse of A (NR x K, full column rank): (A^* A)^+ A^* = Vs (A Vs)^*
  // with Vs = V Lambda^{-1/2} over eigenvalues above 1e-12 of the largest.
  void pinv(const z2* A, int NR, int K, int nb, z2* Pi) {
    if (K <= 0 || NR <= 0) return;
    DBuf G, D, cnt, Vs(zb((int64_t)nb * K * K)), Y(zb((int64_t)nb * NR * K));
    gram_eig(A, NR, K, nb, G, D);
    eig_count(D.as<double>(), K, nb, 1e-12, K, cnt);
    eig_take(G.as<z2>(), K, D.as<double>(), cnt.as<int32_t>(), nb, K, 1, Vs.as<z2>(), (int64_t)K * K, K, 0, nullptr,
             0, 1, nullptr, 0);
    bl.gemm(rocblas_operation_none, rocblas_operation_none, NR, K, K, A, NR, (int64_t)NR * K, Vs.as<z2>(), K,
            (int64_t)K * K, Y.as<z2>(), NR, (int64_t)NR * K, nb);
    bl.gemm(rocblas_operation_none, rocblas_operation_conjugate_transpose, K, NR, K, Vs.as<z2>(), K, (int64_t)K * K,
            Y.as<z2>(), NR, (int64_t)NR * K, Pi, K, (int64_t)K * NR, nb);
  }

  // ------------------------------------------------------------ middle level
  // SVD via random sampling of K_{A,B} for the listed middle-level pairs;
  // results go to store slots slot0 + k.  Returns the ranks.
  std::vector<int32_t> mid_batch(const std::vector<int64_t>& pairs, int64_t slot0, bool store) {
    const int nb = (int)pairs.size();
    const int lB = L - m;
    std::vector<int32_t> aoff(nb), an(nb), boff(nb), bn(nb);
    int Pm = 1, Qm = 1;
    for (int k = 0; k < nb; ++k) {
      const int32_t ia = (int32_t)(pairs[k] / ot.nn(lB)), ib = (int32_t)(pairs[k] % ot.nn(lB));
      aoff[k] = (int32_t)xt.off[m][ia];
      an[k] = (int32_t)xsize(m, ia);
      boff[k] = (int32_t)ot.off[lB][ib];
      bn[k] = (int32_t)osize(lB, ib);
      Pm = std::max(Pm, an[k]);
      Qm = std::max(Qm, bn[k]);
    }
    const int kmax1 = KCAP;
    const double qtol = tol * 1e-2;
    // (1) representative columns: pivoted QR of q randomly selected rows
    std::vector<std::vector<int32_t>> I0(nb);
    std::vector<int32_t> I0c((size_t)nb * q, -1), qb(nb);
    for (int k = 0; k < nb; ++k) {
      const int32_t ia = (int32_t)(pairs[k] / ot.nn(lB)), ib = (int32_t)(pairs[k] % ot.nn(lB));
      std::mt19937_64 rng(mix(mix(o.seed, (uint64_t)ia), (uint64_t)ib) ^ (uint64_t)q);
      I0[k] = sample(rng, an[k], q);
      qb[k] = (int32_t)I0[k].size();
      for (int i = 0; i < qb[k]; ++i) I0c[(size_t)k * q + i] = xcall[aoff[k] + I0[k][i]];
    }
    DBuf dI0 = upload(I0c, st);
    std::vector<EntryDesc> ed(nb);
    // candidate columns: all of B, or a random subset when B is wider than
    // the pivoted-QR kernel takes
    const int Qcand = std::min(Qm, kQrCols);
    std::vector<std::vector<int32_t>> Bc(nb);
    std::vector<int32_t> Bcc((size_t)nb * Qcand, -1), bcn(nb);
    for (int k = 0; k < nb; ++k) {
      if (bn[k] <= Qcand) {
        Bc[k].resize(bn[k]);
        std::iota(Bc[k].begin(), Bc[k].end(), 0);
      } else {
        const int32_t ia = (int32_t)(pairs[k] / ot.nn(lB)), ib = (int32_t)(pairs[k] % ot.nn(lB));
        std::mt19937_64 rng(mix(mix(o.seed ^ 0x2545f491ull, (uint64_t)ia), (uint64_t)ib));
        Bc[k] = sample(rng, bn[k], Qcand);
      }
      bcn[k] = (int32_t)Bc[k].size();
      for (int j = 0; j < bcn[k]; ++j) Bcc[(size_t)k * Qcand + j] = ocall[boff[k] + Bc[k][j]];
    }
    DBuf dBc = upload(Bcc, st);
    DBuf R(zb((int64_t)nb * q * Qcand));
    for (int k = 0; k < nb; ++k) ed[k] = {dI0.as<int32_t>() + (size_t)k * q, dBc.as<int32_t>() + (size_t)k * Qcand, qb[k], bcn[k]};
    entries(ed, q, Qcand, R.as<z2>(), (int64_t)q * Qcand, Qcand, 1, false);
    std::vector<int32_t> J, kc;
    qrcp(R.as<z2>(), (int64_t)q * Qcand, Qcand, qb, bcn, Qcand, kmax1, qtol, J, kc);
    R.release();
    dBc.release();
    for (int k = 0; k < nb; ++k)
      for (int j = 0; j < kc[k]; ++j) J[(size_t)k * kmax1 + j] = Bc[k][J[(size_t)k * kmax1 + j]];
    int KC = 1;
    for (int k = 0; k < nb; ++k) KC = std::max(KC, kc[k]);
    std::vector<std::vector<int32_t>> Jl(nb);
    std::vector<int32_t> Jc((size_t)nb * KC, -1);
    for (int k = 0; k < nb; ++k) {
      Jl[k].assign(J.begin() + (size_t)k * kmax1, J.begin() + (size_t)k * kmax1 + kc[k]);
      std::sort(Jl[k].begin(), Jl[k].end());
      for (int j = 0; j < kc[k]; ++j) Jc[(size_t)k * KC + j] = ocall[boff[k] + Jl[k][j]];
    }
    DBuf dJc = upload(Jc, st);
    // (2) representative rows: pivoted QR of the representative columns
    // (K(A, J)^*: the rows of K(A, J) are the columns of its row-major transpose)
    DBuf C(zb((int64_t)nb * Pm * KC));
    for (int k = 0; k < nb; ++k)
      ed[k] = {d_xcall.as<int32_t>() + aoff[k], dJc.as<int32_t>() + (size_t)k * KC, an[k], kc[k]};
    entries(ed, Pm, KC, C.as<z2>(), (int64_t)Pm * KC, 1, Pm, false);
    std::vector<int32_t> Ip, kr;
    {
      // candidate rows: all of A, or the random rows plus a random subset
      // when A is wider than the pivoted-QR kernel takes
      const int Pc = std::min(Pm, kQrCols);
      std::vector<std::vector<int32_t>> Ac(nb);
      std::vector<int32_t> Acc((size_t)nb * Pc, -1), acn(nb);
      for (int k = 0; k < nb; ++k) {
        if (an[k] <= Pc) {
          Ac[k].resize(an[k]);
          std::iota(Ac[k].begin(), Ac[k].end(), 0);
        } else {
          const int32_t ia = (int32_t)(pairs[k] / ot.nn(lB)), ib = (int32_t)(pairs[k] % ot.nn(lB));
          std::mt19937_64 rng(mix(mix(o.seed ^ 0x9e3779b9ull, (uint64_t)ia), (uint64_t)ib));
          Ac[k] = merge_sorted(I0[k], sample(rng, an[k], Pc - (int32_t)I0[k].size()));
          Ac[k].resize(std::min<size_t>(Ac[k].size(), (size_t)Pc));
        }
        acn[k] = (int32_t)Ac[k].size();
        for (int i = 0; i < acn[k]; ++i) Acc[(size_t)k * Pc + i] = xcall[aoff[k] + Ac[k][i]];
      }
      DBuf dAc = upload(Acc, st);
      DBuf Cq(zb((int64_t)nb * Pc * KC));
      for (int k = 0; k < nb; ++k)
        ed[k] = {dAc.as<int32_t>() + (size_t)k * Pc, dJc.as<int32_t>() + (size_t)k * KC, acn[k], kc[k]};
      entries(ed, Pc, KC, Cq.as<z2>(), (int64_t)Pc * KC, 1, Pc, false);
      qrcp(Cq.as<z2>(), (int64_t)Pc * KC, Pc, kc, acn, Pc, KC, qtol, Ip, kr);
      for (int k = 0; k < nb; ++k)
        for (int i = 0; i < kr[k]; ++i) Ip[(size_t)k * KC + i] = Ac[k][Ip[(size_t)k * KC + i]];
    }
    // index sets: I = the selected representative rows; I_row, I_col contain
    // the representatives plus fresh random indices (overdetermined by q)
    std::vector<std::vector<int32_t>> Ia(nb), Ir(nb), Icl(nb);
    int NI = 1, NR = 1, NC = 1;
    for (int k = 0; k < nb; ++k) {
      const int32_t ia = (int32_t)(pairs[k] / ot.nn(lB)), ib = (int32_t)(pairs[k] % ot.nn(lB));
      std::mt19937_64 rng(mix(mix(o.seed ^ 0x5bd1e995ull, (uint64_t)ia), (uint64_t)ib) ^ (uint64_t)q);
      std::vector<int32_t> sel(Ip.begin() + (size_t)k * KC, Ip.begin() + (size_t)k * KC + kr[k]);
      std::sort(sel.begin(), sel.end());
      Ia[k] = sel;
      Ir[k] = merge_sorted(Ia[k], sample(rng, an[k], kc[k] + q));
      Icl[k] = merge_sorted(Jl[k], sample(rng, bn[k], (int32_t)Ia[k].size() + q));
      NI = std::max(NI, (int)Ia[k].size());
      NR = std::max(NR, (int)Ir[k].size());
      NC = std::max(NC, (int)Icl[k].size());
    }
    if (NI > NICAP) throw DevErr(MBF_ERR_HIP, "middle level: row set above its capacity");
    std::vector<int32_t> Iac((size_t)nb * NI, -1), Irc((size_t)nb * NR, -1), Irl((size_t)nb * NR, -1),
        Icc((size_t)nb * NC, -1), Icloc((size_t)nb * NC, -1), ni(nb), nrr(nb), ncc(nb);
    for (int k = 0; k < nb; ++k) {
      ni[k] = (int32_t)Ia[k].size();
      nrr[k] = (int32_t)Ir[k].size();
      ncc[k] = (int32_t)Icl[k].size();
      for (int i = 0; i < ni[k]; ++i) Iac[(size_t)k * NI + i] = xcall[aoff[k] + Ia[k][i]];
      for (int i = 0; i < nrr[k]; ++i) {
        Irc[(size_t)k * NR + i] = xcall[aoff[k] + Ir[k][i]];
        Irl[(size_t)k * NR + i] = Ir[k][i];
      }
      for (int j = 0; j < ncc[k]; ++j) {
        Icc[(size_t)k * NC + j] = ocall[boff[k] + Icl[k][j]];
        Icloc[(size_t)k * NC + j] = Icl[k][j];
      }
    }
    DBuf dIac = upload(Iac, st), dIrc = upload(Irc, st), dIrl = upload(Irl, st), dIcc = upload(Icc, st),
         dIcl = upload(Icloc, st);
    // (3) orthonormal bases of the representative columns and rows
    DBuf Qc(zb((int64_t)nb * Pm * KC)), Tc(zb((int64_t)nb * KC * KC));
    orth(C.as<z2>(), Pm, KC, nb, Qc.as<z2>(), Tc.as<z2>());
    C.release();
    DBuf Rr(zb((int64_t)nb * Qm * NI)), Qr(zb((int64_t)nb * Qm * NI)), Tr(zb((int64_t)nb * NI * NI));
    for (int k = 0; k < nb; ++k)
      ed[k] = {dIac.as<int32_t>() + (size_t)k * NI, d_ocall.as<int32_t>() + boff[k], ni[k], bn[k]};
    entries(ed, NI, Qm, Rr.as<z2>(), (int64_t)Qm * NI, Qm, 1, true);  // Rr = K(I, B)^*, Qm x NI
    orth(Rr.as<z2>(), Qm, NI, nb, Qr.as<z2>(), Tr.as<z2>());
    Rr.release();
    // (4) middle matrix from the sampled block K(I_row, I_col)
    DBuf Zs(zb((int64_t)nb * NR * NC));
    for (int k = 0; k < nb; ++k)
      ed[k] = {dIrc.as<int32_t>() + (size_t)k * NR, dIcc.as<int32_t>() + (size_t)k * NC, nrr[k], ncc[k]};
    entries(ed, NR, NC, Zs.as<z2>(), (int64_t)NR * NC, 1, NR, false);
    DBuf Qci(zb((int64_t)nb * NR * KC)), Qri(zb((int64_t)nb * NC * NI));
    hipLaunchKernelGGL(k_gather_rows, dim3(gridx((int64_t)NR * KC), nb), dim3(256), 0, st, Qc.as<z2>(),
                       (int64_t)Pm * KC, Pm, dIrl.as<int32_t>(), (int64_t)NR, NR, KC, Qci.as<z2>(), (int64_t)NR * KC);
    hipLaunchKernelGGL(k_gather_rows, dim3(gridx((int64_t)NC * NI), nb), dim3(256), 0, st, Qr.as<z2>(),
                       (int64_t)Qm * NI, Qm, dIcl.as<int32_t>(), (int64_t)NC, NC, NI, Qri.as<z2>(), (int64_t)NC * NI);
    hipck(hipGetLastError(), "k_gather_rows");
    Qc.release();
    Qr.release();
    DBuf P1(zb((int64_t)nb * KC * NR)), P2(zb((int64_t)nb * NI * NC));
    pinv(Qci.as<z2>(), NR, KC, nb, P1.as<z2>());
    pinv(Qri.as<z2>(), NC, NI, nb, P2.as<z2>());
    Qci.release();
    Qri.release();
    DBuf T1(zb((int64_t)nb * KC * NC)), M(zb((int64_t)nb * KC * NI));
    bl.gemm(rocblas_operation_none, rocblas_operation_none, KC, NC, NR, P1.as<z2>(), KC, (int64_t)KC * NR, Zs.as<z2>(),
            NR, (int64_t)NR * NC, T1.as<z2>(), KC, (int64_t)KC * NC, nb);
    bl.gemm(rocblas_operation_none, rocblas_operation_conjugate_transpose, KC, NI, NC, T1.as<z2>(), KC,
            (int64_t)KC * NC, P2.as<z2>(), NI, (int64_t)NI * NC, M.as<z2>(), KC, (int64_t)KC * NI, nb);
    Zs.release();
    T1.release();
    P1.release();
    P2.release();
    // (5) SVD of M: M M^* = U_M Sigma^2 U_M^*
    DBuf G(zb((int64_t)nb * KC * KC)), D((size_t)nb * KC * 8), E((size_t)nb * KC * 8), info((size_t)nb * 4), cnt;
    bl.herk(false, KC, NI, M.as<z2>(), KC, (int64_t)KC * NI, G.as<z2>(), KC, (int64_t)KC * KC, nb);
    bl.heevd(KC, G.as<z2>(), (int64_t)KC * KC, D.as<double>(), E.as<double>(), info.as<int32_t>(), nb);
    std::vector<int32_t> r = eig_count(D.as<double>(), KC, nb, tol * tol, std::min(rmax, RCAP), cnt);
    if (!store) return r;
    DBuf UrS(zb((int64_t)nb * KC * RCAP)), Ur(zb((int64_t)nb * KC * RCAP)), Y(zb((int64_t)nb * NI * RCAP));
    eig_take(G.as<z2>(), KC, D.as<double>(), cnt.as<int32_t>(), nb, RCAP, 2, UrS.as<z2>(), (int64_t)KC * RCAP, KC, 0,
             Ur.as<z2>(), (int64_t)KC * RCAP, KC, mSig.as<double>() + slot0 * RCAP, RCAP);
    // X_u = T_c U_M Sigma (U = K(A, J) X_u = Q_col U_M Sigma), X_v = T_r M^* U_M
    // (V = K(I, B)^* X_v = Q_row V_M Sigma)
    bl.gemm(rocblas_operation_none, rocblas_operation_none, KC, RCAP, KC, Tc.as<z2>(), KC, (int64_t)KC * KC,
            UrS.as<z2>(), KC, (int64_t)KC * RCAP, mXu.as<z2>() + slot0 * KCAP * RCAP, KCAP, (int64_t)KCAP * RCAP, nb);
    bl.gemm(rocblas_operation_conjugate_transpose, rocblas_operation_none, NI, RCAP, KC, M.as<z2>(), KC,
            (int64_t)KC * NI, Ur.as<z2>(), KC, (int64_t)KC * RCAP, Y.as<z2>(), NI, (int64_t)NI * RCAP, nb);
    bl.gemm(rocblas_operation_none, rocblas_operation_none, NI, RCAP, NI, Tr.as<z2>(), NI, (int64_t)NI * NI,
            Y.as<z2>(), NI, (int64_t)NI * RCAP, mXv.as<z2>() + slot0 * NICAP * RCAP, NICAP, (int64_t)NICAP * RCAP,
            nb);
    hipck(hipMemcpy2DAsync(mJ.as<int32_t>() + slot0 * KCAP, (size_t)KCAP * 4, dJc.p, (size_t)KC * 4, (size_t)KC * 4,
                           (size_t)nb, hipMemcpyDeviceToDevice, st),
          "copy J");
    hipck(hipMemcpy2DAsync(mI.as<int32_t>() + slot0 * NICAP, (size_t)NICAP * 4, dIac.p, (size_t)NI * 4,
                           (size_t)NI * 4, (size_t)nb, hipMemcpyDeviceToDevice, st),
          "copy I");
    hipck(hipStreamSynchronize(st), "middle batch");
    for (int k = 0; k < nb; ++k) {
      m_kc[slot0 + k] = kc[k];
      m_ni[slot0 + k] = ni[k];
    }
    return r;
  }

  size_t mid_bytes_per_pair(int Pm, int Qm) const {
    const int64_t KC = KCAP, NI = NICAP, NR = NICAP + KCAP + q, NC = KCAP + NICAP + q;
    const int64_t c = (int64_t)q * Qm + 4 * (int64_t)Pm * KC + 4 * (int64_t)Qm * NI + NR * NC + 2 * NR * KC +
                      2 * NC * NI + NR * KC + NC * NI + KC * NC + KC * NI + 6 * KC * KC + 6 * NI * NI +
                      3 * KC * RCAP + NI * RCAP;
    return (size_t)c * sizeof(z2);
  }

  int pair_min(int64_t p) const {
    const int lB = L - m;
    return (int)std::min(xsize(m, (int32_t)(p / ot.nn(lB))), osize(lB, (int32_t)(p % ot.nn(lB))));
  }

  void middle() {
    const int lB = L - m;
    const int64_t np = (int64_t)xt.nn(m) * ot.nn(lB);
    int Pm = 1, Qm = 1;
    for (int32_t i = 0; i < xt.nn(m); ++i) Pm = std::max<int>(Pm, (int)xsize(m, i));
    for (int32_t i = 0; i < ot.nn(lB); ++i) Qm = std::max<int>(Qm, (int)osize(lB, i));
    // q random rows (at most |A|); at most min(q, |B|, max_rank + oversample)
    // representative columns
    const int qcap = Pm;
    auto set_caps = [&](int qq) {
      q = std::min(qq, qcap);
      KCAP = std::max(1, std::min(std::min(q, Qm), rmax + os));
      NICAP = KCAP;
      RCAP = KCAP;
    };
    // sample size from a spread of probe pairs: doubled until the ranks found
    // stay below q - oversample
    std::vector<int64_t> probe;
    const int64_t nprobe = std::min<int64_t>(np, 32);
    for (int64_t k = 0; k < nprobe; ++k) probe.push_back(k * np / nprobe);
    set_caps(std::max(32, 2 * os + 16));
    for (;;) {
      std::vector<int32_t> r = mid_batch(probe, 0, false);
      // a rank that reaches min(|A|, |B|) cannot grow with more samples
      int rm = 0;
      bool more = false;
      for (size_t k = 0; k < r.size(); ++k) {
        rm = std::max(rm, r[k]);
        more = more || (r[k] + os > q && r[k] < pair_min(probe[k]));
      }
      if (!more || q >= qcap || rm >= rmax) {
        set_caps(std::max(q, rm + 2 * os));
        break;
      }
      set_caps(2 * q);
    }
    rank[m].assign(np, 0);
    for (;;) {
      m_kc.assign(np, 0);
      m_ni.assign(np, 0);
      mJ.alloc((size_t)np * KCAP * 4);
      mI.alloc((size_t)np * NICAP * 4);
      mXu.alloc(zb(np * KCAP * RCAP));
      mXv.alloc(zb(np * NICAP * RCAP));
      mSig.alloc((size_t)np * RCAP * 8);
      hipck(hipMemsetAsync(mJ.p, 0xff, mJ.bytes, st), "memset");
      hipck(hipMemsetAsync(mI.p, 0xff, mI.bytes, st), "memset");
      hipck(hipMemsetAsync(mXu.p, 0, mXu.bytes, st), "memset");
      hipck(hipMemsetAsync(mXv.p, 0, mXv.bytes, st), "memset");
      const int64_t per = std::max<int64_t>(1, (int64_t)(budget / std::max<size_t>(1, mid_bytes_per_pair(Pm, Qm))));
      const int64_t nbatch = std::min<int64_t>(std::min<int64_t>(per, np), 65535);
      bool redo = false;
      for (int64_t p0 = 0; p0 < np && !redo; p0 += nbatch) {
        const int64_t p1 = std::min(np, p0 + nbatch);
        std::vector<int64_t> pl(p1 - p0);
        std::iota(pl.begin(), pl.end(), p0);
        std::vector<int32_t> r = mid_batch(pl, p0, true);
        for (int64_t k = 0; k < p1 - p0; ++k) {
          rank[m][p0 + k] = r[k];
          if (r[k] + os > q && q < qcap && r[k] < rmax && r[k] < pair_min(p0 + k)) redo = true;
        }
        if (verbose()) {
          char buf[128];
          std::snprintf(buf, sizeof(buf), "middle level %lld/%lld pairs (q = %d)", (long long)p1, (long long)np, q);
          log(buf);
        }
      }
      if (!redo) break;
      set_caps(2 * q);
      log("middle level: a rank reached the sample size; sampling again with twice as many rows");
    }
  }

  // Regenerate U^h (forward=true: K(A, J) X_u, |A| x RCAP) or V^h
  // (K(I, B)^* X_v, |B| x RCAP) for the listed middle pairs into `out`
  // (one matrix per listed pair, ld = rows).
  int regen(const std::vector<int64_t>& pl, bool u, DBuf& out) {
    const int lB = L - m;
    const int nb = (int)pl.size();
    int P = 1;
    for (int64_t p : pl) {
      const int32_t ia = (int32_t)(p / ot.nn(lB)), ib = (int32_t)(p % ot.nn(lB));
      P = std::max<int>(P, (int)(u ? xsize(m, ia) : osize(lB, ib)));
    }
    const int KK = u ? KCAP : NICAP;
    DBuf E(zb((int64_t)nb * P * KK));
    std::vector<EntryDesc> ed(nb);
    for (int k = 0; k < nb; ++k) {
      const int64_t p = pl[k];
      const int32_t ia = (int32_t)(p / ot.nn(lB)), ib = (int32_t)(p % ot.nn(lB));
      if (u)
        ed[k] = {d_xcall.as<int32_t>() + xt.off[m][ia], mJ.as<int32_t>() + p * KCAP, (int32_t)xsize(m, ia), m_kc[p]};
      else
        ed[k] = {mI.as<int32_t>() + p * NICAP, d_ocall.as<int32_t>() + ot.off[lB][ib], m_ni[p], (int32_t)osize(lB, ib)};
    }
    if (u)
      entries(ed, P, KK, E.as<z2>(), (int64_t)P * KK, 1, P, false);
    else
      entries(ed, KK, P, E.as<z2>(), (int64_t)P * KK, P, 1, true);
    out.alloc(zb((int64_t)nb * P * RCAP));
    // X_u / X_v of the listed pairs, gathered contiguously
    DBuf X(zb((int64_t)nb * KK * RCAP));
    const z2* base = u ? mXu.as<z2>() : mXv.as<z2>();
    for (int k = 0; k < nb;) {
      int k1 = k + 1;
      while (k1 < nb && pl[k1] == pl[k1 - 1] + 1) ++k1;
      hipck(hipMemcpyAsync(X.as<z2>() + (int64_t)k * KK * RCAP, base + pl[k] * KK * RCAP,
                           (size_t)(k1 - k) * KK * RCAP * sizeof(z2), hipMemcpyDeviceToDevice, st),
            "copy X");
      k = k1;
    }
    bl.gemm(rocblas_operation_none, rocblas_operation_none, P, RCAP, KK, E.as<z2>(), P, (int64_t)P * KK, X.as<z2>(), KK,
            (int64_t)KK * RCAP, out.as<z2>(), P, (int64_t)P * RCAP, nb);
    return P;
  }

  // ------------------------------------------------------------- recursions
  // One W per entry of `gds` (P x Kc after the merge); returns the ranks,
  // the next-level matrices (P x R each, in `next_buf`) and the source of
  // the stage-block pieces.
  struct Trunc {
    bool wide = false;
    int R = 0, P = 0, Kc = 0;
    DBuf unext, gsrc;
    int gld = 1;
    std::vector<int32_t> r;
  };

  // Truncated SVD of every merged block W (P x Kc after the merge), form 2:
  // W ~ U_next G with U_next = U_0 Sigma.  When the expected rank is well
  // below min(P, Kc), the range of W is first captured by a Gaussian sketch
  // Y = W Omega with `over` extra columns (randomized range finder), and the
  // SVD is taken of Q^* W for an orthonormal basis Q of Y; a member whose
  // rank comes within a few columns of the sketch width sends the batch back
  // to the exact Gram eigendecomposition.
  Trunc truncate(const std::vector<GatherDesc>& gds, int P, int Kc, int r_est) {
    Trunc t;
    const int nb = (int)gds.size();
    t.P = P;
    t.Kc = Kc;
    t.r.assign(nb, 0);
    if (Kc <= 0 || P <= 0) return t;
    DBuf W(zb((int64_t)nb * P * Kc));
    {
      DBuf dg = upload(gds, st);
      hipLaunchKernelGGL(k_gather, dim3(gridx((int64_t)P * Kc), nb), dim3(256), 0, st, dg.as<GatherDesc>(), P, Kc,
                         W.as<z2>(), (int64_t)P * Kc);
      hipck(hipGetLastError(), "k_gather");
      hipck(hipStreamSynchronize(st), "k_gather");
    }
    g_tm.mark(st, T_SMALL);
    const int d = std::min(P, Kc);
    const int over = 48;
    const int l = std::min(d, std::max(r_est, 1) + over);
    if (l * 5 < d * 3 && sketch(W.as<z2>(), nb, P, Kc, l, t)) return t;
    t.wide = P < Kc;
    const int cap = std::min(rmax, d);
    DBuf G(zb((int64_t)nb * d * d)), D((size_t)nb * d * 8), E((size_t)nb * d * 8), info((size_t)nb * 4), cnt;
    if (t.wide)
      bl.herk(false, P, Kc, W.as<z2>(), P, (int64_t)P * Kc, G.as<z2>(), P, (int64_t)P * P, nb);
    else
      bl.herk(true, Kc, P, W.as<z2>(), P, (int64_t)P * Kc, G.as<z2>(), Kc, (int64_t)Kc * Kc, nb);
    bl.heevd(d, G.as<z2>(), (int64_t)d * d, D.as<double>(), E.as<double>(), info.as<int32_t>(), nb);
    t.r = eig_count(D.as<double>(), d, nb, tol * tol, cap, cnt);
    t.R = 0;
    for (int v : t.r) t.R = std::max(t.R, v);
    if (t.R == 0) return t;
    const int R = t.R;
    t.unext.alloc(zb((int64_t)nb * P * R));
    if (!t.wide) {
      // W^* W = V Lambda V^*:  U_next = W V_r,  block piece = V_r^*
      t.gsrc.alloc(zb((int64_t)nb * Kc * R));
      eig_take(G.as<z2>(), d, D.as<double>(), cnt.as<int32_t>(), nb, R, 0, t.gsrc.as<z2>(), (int64_t)Kc * R, Kc, 0,
               nullptr, 0, 1, nullptr, 0);
      bl.gemm(rocblas_operation_none, rocblas_operation_none, P, R, Kc, W.as<z2>(), P, (int64_t)P * Kc,
              t.gsrc.as<z2>(), Kc, (int64_t)Kc * R, t.unext.as<z2>(), P, (int64_t)P * R, nb);
      t.gld = Kc;
    } else {
      // W W^* = U Lambda U^*:  U_next = U_r Sigma_r,  block piece = Sigma_r^{-1} U_r^* W
      DBuf Ub(zb((int64_t)nb * P * R));
      eig_take(G.as<z2>(), d, D.as<double>(), cnt.as<int32_t>(), nb, R, 2, t.unext.as<z2>(), (int64_t)P * R, P, 1,
               Ub.as<z2>(), (int64_t)P * R, P, nullptr, 0);
      t.gsrc.alloc(zb((int64_t)nb * R * Kc));
      bl.gemm(rocblas_operation_conjugate_transpose, rocblas_operation_none, R, Kc, P, Ub.as<z2>(), P, (int64_t)P * R,
              W.as<z2>(), P, (int64_t)P * Kc, t.gsrc.as<z2>(), R, (int64_t)R * Kc, nb);
      t.gld = R;
    }
    hipck(hipStreamSynchronize(st), "truncate");
    return t;
  }

  // Randomized range finder path of truncate (see there).  Returns false
  // when some member's rank reaches the sketch width minus 4.
  bool sketch(const z2* W, int nb, int P, int Kc, int l, Trunc& t) {
    std::vector<z2> om((size_t)Kc * l);
    std::mt19937_64 rng(mix(o.seed ^ 0x85ebca6bull, (uint64_t)Kc * 131 + (uint64_t)l));
    std::normal_distribution<double> nd(0.0, std::sqrt(0.5));
    for (auto& v : om) v = make_double2(nd(rng), nd(rng));
    DBuf dom = upload(om, st);
    DBuf Y(zb((int64_t)nb * P * l)), Q(zb((int64_t)nb * P * l)), Ty(zb((int64_t)nb * l * l)), B(zb((int64_t)nb * l * Kc));
    bl.gemm(rocblas_operation_none, rocblas_operation_none, P, l, Kc, W, P, (int64_t)P * Kc, dom.as<z2>(), Kc, 0,
            Y.as<z2>(), P, (int64_t)P * l, nb);
    orth(Y.as<z2>(), P, l, nb, Q.as<z2>(), Ty.as<z2>());
    Y.release();
    bl.gemm(rocblas_operation_conjugate_transpose, rocblas_operation_none, l, Kc, P, Q.as<z2>(), P, (int64_t)P * l, W,
            P, (int64_t)P * Kc, B.as<z2>(), l, (int64_t)l * Kc, nb);
    DBuf G(zb((int64_t)nb * l * l)), D((size_t)nb * l * 8), E((size_t)nb * l * 8), info((size_t)nb * 4), cnt;
    bl.herk(false, l, Kc, B.as<z2>(), l, (int64_t)l * Kc, G.as<z2>(), l, (int64_t)l * l, nb);
    bl.heevd(l, G.as<z2>(), (int64_t)l * l, D.as<double>(), E.as<double>(), info.as<int32_t>(), nb);
    std::vector<int32_t> r = eig_count(D.as<double>(), l, nb, tol * tol, std::min(rmax, l), cnt);
    int R = 0;
    for (int v : r) {
      if (v > l - 4 && v < rmax) return false;
      R = std::max(R, v);
    }
    t.r = r;
    t.R = R;
    t.wide = true;  // block piece stored as R x Kc
    if (R == 0) return true;
    DBuf Ua(zb((int64_t)nb * l * R)), Ub(zb((int64_t)nb * l * R));
    eig_take(G.as<z2>(), l, D.as<double>(), cnt.as<int32_t>(), nb, R, 2, Ua.as<z2>(), (int64_t)l * R, l, 1, Ub.as<z2>(),
             (int64_t)l * R, l, nullptr, 0);
    // U_next = Q U_r Sigma_r,  block piece = Sigma_r^{-1} U_r^* B  (B = Q^* W)
    t.unext.alloc(zb((int64_t)nb * P * R));
    bl.gemm(rocblas_operation_none, rocblas_operation_none, P, R, l, Q.as<z2>(), P, (int64_t)P * l, Ua.as<z2>(), l,
            (int64_t)l * R, t.unext.as<z2>(), P, (int64_t)P * R, nb);
    t.gsrc.alloc(zb((int64_t)nb * R * Kc));
    bl.gemm(rocblas_operation_conjugate_transpose, rocblas_operation_none, R, Kc, l, Ub.as<z2>(), l, (int64_t)l * R,
            B.as<z2>(), l, (int64_t)l * Kc, t.gsrc.as<z2>(), R, (int64_t)R * Kc, nb);
    t.gld = R;
    hipck(hipStreamSynchronize(st), "sketch");
    return true;
  }

  // Write the pieces of a batch of blocks of `stage` into a new piece of
  // that stage (every precision of the mask).
  void pack(int stage, const std::vector<PackDesc>& pds, int64_t elems) {
    Piece pc;
    pc.elems = elems;
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p)) || elems == 0) continue;
      const size_t es = p == MBF_C128 ? 16 : 8;
      DBuf b((size_t)elems * es);
      pc.p[p] = b.take();
    }
    pieces[stage].push_back(pc);
    if (elems == 0 || pds.empty()) return;
    int64_t mx = 1;
    for (auto& d : pds) mx = std::max<int64_t>(mx, (int64_t)d.ni * d.nj);
    DBuf dp = upload(pds, st);
    hipLaunchKernelGGL(k_pack, dim3(gridx(mx), (unsigned)pds.size()), dim3(256), 0, st, dp.as<PackDesc>(),
                       static_cast<z2*>(pc.p[MBF_C128]), static_cast<float2*>(pc.p[MBF_C64]),
                       static_cast<ushort4*>(pc.p[MBF_C64_SPLIT_BF16]));
    hipck(hipGetLastError(), "k_pack");
    hipck(hipStreamSynchronize(st), "k_pack");
    g_tm.mark(st, T_SMALL);
  }

  size_t w_bytes(int P, int Kc) const {
    const int64_t d = std::min(P, Kc), R = std::min<int64_t>(d, rmax);
    return (size_t)((int64_t)P * Kc + d * d + 2 * (int64_t)P * R + (int64_t)Kc * R + R * Kc) * sizeof(z2) + 64;
  }

  // U recursion (Section 2.4.1): stage s -> s+1, s = m .. L-1.  Parents
  // (A at X-level s, B' at Omega-level L-s-1) in block order; W_t for every
  // X child A_t of A; U^{s+1}_{A_t,B'} and G^s_{A_t,B'}.
  void u_side() {
    Mats cur;
    for (int s = m; s < L; ++s) {
      const int lo = L - s - 1;
      const int64_t nparent = (int64_t)xt.nn(s) * ot.nn(lo);
      Mats next;
      next.reset((size_t)xt.nn(s + 1) * ot.nn(lo));
      rank[s + 1].assign((size_t)xt.nn(s + 1) * ot.nn(lo), 0);
      int Pmax = 1, Kmax = 1;
      for (int32_t i = 0; i < xt.nn(s + 1); ++i) Pmax = std::max<int>(Pmax, (int)xsize(s + 1, i));
      for (int32_t ia = 0; ia < xt.nn(s); ++ia)
        for (int32_t ibp = 0; ibp < ot.nn(lo); ++ibp) {
          int K = 0;
          for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib) K += rank[s][pair(s, ia, ib)];
          Kmax = std::max(Kmax, K);
        }
      size_t per = 4 * w_bytes(Pmax, Kmax);
      if (s == m) per += 4 * (size_t)xsize(m, 0) * (KCAP + 2 * RCAP) * sizeof(z2);
      const int r_in_max = *std::max_element(rank[s].begin(), rank[s].end());
      const int64_t pbatch = std::max<int64_t>(1, std::min<int64_t>((int64_t)(budget / per), 16383));
      for (int64_t q0 = 0; q0 < nparent; q0 += pbatch) {
        const int64_t q1 = std::min(nparent, q0 + pbatch);
        DBuf regen_buf;
        std::vector<int64_t> regen_pairs;
        int regen_P = 0;
        if (s == m) {
          for (int64_t pp = q0; pp < q1; ++pp) {
            const int32_t ia = (int32_t)(pp / ot.nn(lo)), ibp = (int32_t)(pp % ot.nn(lo));
            for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib) regen_pairs.push_back(pair(s, ia, ib));
          }
          regen_P = regen(regen_pairs, true, regen_buf);
        }
        auto src_of = [&](int64_t p, const z2*& ptr, int32_t& ld) {
          if (s == m) {
            const int64_t k = std::lower_bound(regen_pairs.begin(), regen_pairs.end(), p) - regen_pairs.begin();
            ptr = regen_buf.as<z2>() + k * (int64_t)regen_P * RCAP;
            ld = regen_P;
          } else {
            ptr = cur.ptr[p];
            ld = cur.ld[p];
          }
        };
        std::vector<GatherDesc> gds;
        std::vector<std::pair<int64_t, int32_t>> wmap;  // (parent, child X node)
        int P = 1, Kc = 1;
        for (int64_t pp = q0; pp < q1; ++pp) {
          const int32_t ia = (int32_t)(pp / ot.nn(lo)), ibp = (int32_t)(pp % ot.nn(lo));
          for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it) {
            GatherDesc g{};
            int K = 0, sl = 0;
            for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib, ++sl) {
              const int64_t p = pair(s, ia, ib);
              src_of(p, g.src[sl], g.ld[sl]);
              g.nc[sl] = rank[s][p];
              K += g.nc[sl];
            }
            for (; sl < 4; ++sl) {
              g.src[sl] = g.src[0];
              g.ld[sl] = 1;
              g.nc[sl] = 0;
            }
            g.row0 = (int32_t)(xt.off[s + 1][it] - xt.off[s][ia]);
            g.nrow = (int32_t)xsize(s + 1, it);
            P = std::max<int>(P, g.nrow);
            Kc = std::max(Kc, K);
            gds.push_back(g);
            wmap.push_back({pp, it});
          }
        }
        Trunc t = truncate(gds, P, Kc, r_in_max);
        const int nw = (int)gds.size();
        for (int w = 0; w < nw; ++w) {
          const int32_t ibp = (int32_t)(wmap[w].first % ot.nn(lo));
          const int64_t pn = pair(s + 1, wmap[w].second, ibp);
          rank[s + 1][pn] = t.r[w];
          next.ptr[pn] = t.R > 0 ? t.unext.as<z2>() + (int64_t)w * P * t.R : nullptr;
          next.ld[pn] = P;
        }
        // stage-s blocks of these parents: rows grouped by the X children
        std::vector<PackDesc> pds;
        int64_t off = 0;
        int w = 0;
        for (int64_t pp = q0; pp < q1; ++pp) {
          const int32_t ia = (int32_t)(pp / ot.nn(lo)), ibp = (int32_t)(pp % ot.nn(lo));
          int32_t K = 0, M = 0;
          for (int32_t ib = ot.cfirst[lo][ibp]; ib < ot.cfirst[lo][ibp + 1]; ++ib) K += rank[s][pair(s, ia, ib)];
          for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it) M += rank[s + 1][pair(s + 1, it, ibp)];
          int32_t ms = 0;
          for (int32_t it = xt.cfirst[s][ia]; it < xt.cfirst[s][ia + 1]; ++it, ++w) {
            const int32_t r = t.r[w];
            if (r > 0 && K > 0) {
              PackDesc d{};
              d.src = t.gsrc.as<z2>() + (int64_t)w * (t.wide ? (int64_t)t.R * Kc : (int64_t)Kc * t.R);
              d.dst = off;
              d.ld = t.gld;
              d.ni = r;
              d.nj = K;
              d.M = M;
              d.r0 = ms;
              d.c0 = 0;
              d.tconj = t.wide ? 0 : 1;
              pds.push_back(d);
            }
            ms += r;
          }
          off += (int64_t)M * K;
        }
        pack(s, pds, off);
        if (t.R > 0) next.bufs.push_back(std::move(t.unext));
        if (verbose()) {
          char buf[160];
          std::snprintf(buf, sizeof(buf), "U recursion stage %d: %lld/%lld blocks (W %d x %d)", s, (long long)q1,
                        (long long)nparent, P, Kc);
          log(buf);
        }
      }
      cur = std::move(next);
    }
    if (m == L) {
      // depth 0: the middle level is the leaf level
      std::vector<int64_t> pl = {0};
      cur.reset(1);
      cur.bufs.emplace_back();
      const int P = regen(pl, true, cur.bufs.back());
      cur.ptr[0] = cur.bufs.back().as<z2>();
      cur.ld[0] = P;
    }
    u_leaves = std::move(cur);
  }

  // V recursion (Section 2.4.2, mirror image): stage s -> s-1, s = m .. 1.
  // Parents (A at X-level s-1, B at Omega-level L-s) in block order; W_c for
  // every Omega child B_c of B; V^{s-1}_{A,B_c} and H^{s-1}_{B_c,A}.
  void v_side() {
    Mats cur;
    for (int s = m; s >= 1; --s) {
      const int lb = L - s;  // Omega level of B
      const int64_t nparent = (int64_t)xt.nn(s - 1) * ot.nn(lb);
      Mats next;
      next.reset((size_t)xt.nn(s - 1) * ot.nn(lb + 1));
      rank[s - 1].assign((size_t)xt.nn(s - 1) * ot.nn(lb + 1), 0);
      int Pmax = 1, Kmax = 1;
      for (int32_t i = 0; i < ot.nn(lb + 1); ++i) Pmax = std::max<int>(Pmax, (int)osize(lb + 1, i));
      for (int32_t iap = 0; iap < xt.nn(s - 1); ++iap)
        for (int32_t ib = 0; ib < ot.nn(lb); ++ib) {
          int K = 0;
          for (int32_t it = xt.cfirst[s - 1][iap]; it < xt.cfirst[s - 1][iap + 1]; ++it) K += rank[s][pair(s, it, ib)];
          Kmax = std::max(Kmax, K);
        }
      size_t per = 4 * w_bytes(Pmax, Kmax);
      if (s == m) per += 4 * (size_t)osize(lb, 0) * (NICAP + 2 * RCAP) * sizeof(z2);
      const int r_in_max = *std::max_element(rank[s].begin(), rank[s].end());
      const int64_t pbatch = std::max<int64_t>(1, std::min<int64_t>((int64_t)(budget / per), 16383));
      for (int64_t q0 = 0; q0 < nparent; q0 += pbatch) {
        const int64_t q1 = std::min(nparent, q0 + pbatch);
        DBuf regen_buf;
        std::vector<int64_t> regen_pairs;
        int regen_P = 0;
        if (s == m) {
          for (int64_t pp = q0; pp < q1; ++pp) {
            const int32_t iap = (int32_t)(pp / ot.nn(lb)), ib = (int32_t)(pp % ot.nn(lb));
            for (int32_t it = xt.cfirst[s - 1][iap]; it < xt.cfirst[s - 1][iap + 1]; ++it)
              regen_pairs.push_back(pair(s, it, ib));
          }
          std::sort(regen_pairs.begin(), regen_pairs.end());
          regen_pairs.erase(std::unique(regen_pairs.begin(), regen_pairs.end()), regen_pairs.end());
          regen_P = regen(regen_pairs, false, regen_buf);
        }
        auto src_of = [&](int64_t p, const z2*& ptr, int32_t& ld) {
          if (s == m) {
            const int64_t k = std::lower_bound(regen_pairs.begin(), regen_pairs.end(), p) - regen_pairs.begin();
            ptr = regen_buf.as<z2>() + k * (int64_t)regen_P * RCAP;
            ld = regen_P;
          } else {
            ptr = cur.ptr[p];
            ld = cur.ld[p];
          }
        };
        std::vector<GatherDesc> gds;
        std::vector<std::pair<int64_t, int32_t>> wmap;  // (parent, child Omega node)
        int P = 1, Kc = 1;
        for (int64_t pp = q0; pp < q1; ++pp) {
          const int32_t iap = (int32_t)(pp / ot.nn(lb)), ib = (int32_t)(pp % ot.nn(lb));
          for (int32_t ibc = ot.cfirst[lb][ib]; ibc < ot.cfirst[lb][ib + 1]; ++ibc) {
            GatherDesc g{};
            int K = 0, sl = 0;
            for (int32_t it = xt.cfirst[s - 1][iap]; it < xt.cfirst[s - 1][iap + 1]; ++it, ++sl) {
              const int64_t p = pair(s, it, ib);
              src_of(p, g.src[sl], g.ld[sl]);
              g.nc[sl] = rank[s][p];
              K += g.nc[sl];
            }
            for (; sl < 4; ++sl) {
              g.src[sl] = g.src[0];
              g.ld[sl] = 1;
              g.nc[sl] = 0;
            }
            g.row0 = (int32_t)(ot.off[lb + 1][ibc] - ot.off[lb][ib]);
            g.nrow = (int32_t)osize(lb + 1, ibc);
            P = std::max<int>(P, g.nrow);
            Kc = std::max(Kc, K);
            gds.push_back(g);
            wmap.push_back({pp, ibc});
          }
        }
        Trunc t = truncate(gds, P, Kc, r_in_max);
        const int nw = (int)gds.size();
        for (int w = 0; w < nw; ++w) {
          const int32_t iap = (int32_t)(wmap[w].first / ot.nn(lb));
          const int64_t pn = pair(s - 1, iap, wmap[w].second);
          rank[s - 1][pn] = t.r[w];
          next.ptr[pn] = t.R > 0 ? t.unext.as<z2>() + (int64_t)w * P * t.R : nullptr;
          next.ld[pn] = P;
        }
        // stage-(s-1) blocks of these parents: columns grouped by the Omega children
        std::vector<PackDesc> pds;
        int64_t off = 0;
        int w = 0;
        for (int64_t pp = q0; pp < q1; ++pp) {
          const int32_t iap = (int32_t)(pp / ot.nn(lb)), ib = (int32_t)(pp % ot.nn(lb));
          int32_t K = 0, M = 0;
          for (int32_t ibc = ot.cfirst[lb][ib]; ibc < ot.cfirst[lb][ib + 1]; ++ibc) K += rank[s - 1][pair(s - 1, iap, ibc)];
          for (int32_t it = xt.cfirst[s - 1][iap]; it < xt.cfirst[s - 1][iap + 1]; ++it) M += rank[s][pair(s, it, ib)];
          int32_t ks = 0;
          for (int32_t ibc = ot.cfirst[lb][ib]; ibc < ot.cfirst[lb][ib + 1]; ++ibc, ++w) {
            const int32_t r = t.r[w];
            if (r > 0 && M > 0) {
              PackDesc d{};
              d.src = t.gsrc.as<z2>() + (int64_t)w * (t.wide ? (int64_t)t.R * Kc : (int64_t)Kc * t.R);
              d.dst = off;
              d.ld = t.gld;
              d.ni = M;
              d.nj = r;
              d.M = M;
              d.r0 = 0;
              d.c0 = ks;
              d.tconj = t.wide ? 1 : 0;
              pds.push_back(d);
            }
            ks += r;
          }
          off += (int64_t)M * K;
        }
        pack(s - 1, pds, off);
        if (t.R > 0) next.bufs.push_back(std::move(t.unext));
        if (verbose()) {
          char buf[160];
          std::snprintf(buf, sizeof(buf), "V recursion stage %d: %lld/%lld blocks (W %d x %d)", s - 1, (long long)q1,
                        (long long)nparent, P, Kc);
          log(buf);
        }
      }
      cur = std::move(next);
    }
    if (m == 0) {
      // no V recursion: the middle level pairs (X root, Omega leaf) are the leaves
      const int64_t np = ot.nn(L);
      std::vector<int64_t> pl(np);
      std::iota(pl.begin(), pl.end(), 0);
      cur.reset(np);
      cur.bufs.emplace_back();
      const int P = regen(pl, false, cur.bufs.back());
      for (int64_t k = 0; k < np; ++k) {
        cur.ptr[k] = cur.bufs.back().as<z2>() + k * (int64_t)P * RCAP;
        cur.ld[k] = P;
      }
    }
    v_leaves = std::move(cur);
  }

  // --------------------------------------------------------------- assembly
  void assemble(const int64_t* idx_map, DevPart& P) {
    std::vector<int64_t> blk_off;
    Error e = layout_part(xt, ot, L, m, rank, idx_map, P, &blk_off);
    if (e.st != MBF_OK) throw DevErr(e.st, e.msg);
    // stages: join the pieces into one allocation per stage and precision
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      P.prec[p].present = true;
      P.prec[p].Wst.assign(L, nullptr);
    }
    for (int s = 0; s < L; ++s) {
      const int64_t se = ((s + 1 < L) ? P.w_stage_off[s + 1] : P.w_elems) - P.w_stage_off[s];
      int64_t tot = 0;
      for (auto& pc : pieces[s]) tot += pc.elems;
      if (tot != se) throw DevErr(MBF_ERR_HIP, "device builder: stage " + std::to_string(s) + " size mismatch");
      for (int p = 0; p < kNumPrec; ++p) {
        if (!(mask & (1u << p)) || se == 0) continue;
        const size_t es = p == MBF_C128 ? 16 : 8;
        DBuf b((size_t)se * es);
        int64_t o = 0;
        for (auto& pc : pieces[s]) {
          if (pc.elems)
            hipck(hipMemcpyAsync((char*)b.p + (size_t)o * es, pc.p[p], (size_t)pc.elems * es, hipMemcpyDeviceToDevice, st),
                  "join stage");
          o += pc.elems;
        }
        hipck(hipStreamSynchronize(st), "join stage");
        for (auto& pc : pieces[s])
          if (pc.p[p]) {
            (void)hipFree(pc.p[p]);
            pc.p[p] = nullptr;
          }
        P.prec[p].bytes += b.bytes;
        P.prec[p].Wst[s] = b.p;
        P.prec[p].Walloc.push_back(b.take());
      }
    }
    // leaves
    auto leaves = [&](const Mats& mats, bool u_leaf) {
      const int nleaf = u_leaf ? xt.nn(L) : ot.nn(L);
      std::vector<LeafPack> lp;
      int64_t fo = 0, mx = 1;
      for (int32_t i = 0; i < nleaf; ++i) {
        const int64_t pr = u_leaf ? pair(L, i, 0) : pair(0, 0, i);
        const int32_t np = (int32_t)(u_leaf ? xsize(L, i) : osize(L, i));
        const int32_t r = u_leaf ? rank[L][pr] : rank[0][pr];
        if (np > 0 && r > 0) lp.push_back(LeafPack{mats.ptr[pr], fo, mats.ld[pr], np, r, 0});
        fo += (int64_t)np * r;
        mx = std::max<int64_t>(mx, (int64_t)np * r);
      }
      if (fo != (u_leaf ? P.u_elems : P.v_elems)) throw DevErr(MBF_ERR_HIP, "device builder: leaf size mismatch");
      DBuf d128, d64;
      if (mask & (1u << MBF_C128)) d128.alloc(zb(fo));
      if (mask & ((1u << MBF_C64) | (1u << MBF_C64_SPLIT_BF16))) d64.alloc((size_t)std::max<int64_t>(fo, 1) * 8);
      if (!lp.empty()) {
        DBuf dl = upload(lp, st);
        hipLaunchKernelGGL(k_pack_leaf, dim3(gridx(mx), (unsigned)lp.size()), dim3(256), 0, st, dl.as<LeafPack>(),
                           d128.as<z2>(), d64.as<float2>());
        hipck(hipGetLastError(), "k_pack_leaf");
        hipck(hipStreamSynchronize(st), "k_pack_leaf");
      }
      for (int p = 0; p < kNumPrec; ++p) {
        if (!(mask & (1u << p))) continue;
        DBuf& src = p == MBF_C128 ? d128 : d64;
        DBuf cp(src.bytes);
        hipck(hipMemcpyAsync(cp.p, src.p, src.bytes, hipMemcpyDeviceToDevice, st), "leaf copy");
        hipck(hipStreamSynchronize(st), "leaf copy");
        P.prec[p].bytes += cp.bytes;
        (u_leaf ? P.prec[p].UL : P.prec[p].V0) = cp.take();
      }
    };
    leaves(u_leaves, true);
    leaves(v_leaves, false);
    // middle scaling
    const int64_t np = (int64_t)rank[m].size();
    std::vector<int64_t> roff(np);
    int64_t acc = 0;
    for (int64_t k = 0; k < np; ++k) {
      roff[k] = acc;
      acc += rank[m][k];
    }
    DBuf dr = upload(rank[m], st), dro = upload(roff, st);
    DBuf s128, s32;
    if (mask & (1u << MBF_C128)) s128.alloc((size_t)std::max<int64_t>(acc, 1) * 8);
    if (mask & ((1u << MBF_C64) | (1u << MBF_C64_SPLIT_BF16))) s32.alloc((size_t)std::max<int64_t>(acc, 1) * 4);
    hipLaunchKernelGGL(k_pack_s, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, mSig.as<double>(), (int64_t)RCAP,
                       dr.as<int32_t>(), dro.as<int64_t>(), (int)np, s128.as<double>(), s32.as<float>());
    hipck(hipGetLastError(), "k_pack_s");
    hipck(hipStreamSynchronize(st), "k_pack_s");
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(mask & (1u << p))) continue;
      DBuf& src = p == MBF_C128 ? s128 : s32;
      DBuf cp(src.bytes);
      hipck(hipMemcpyAsync(cp.p, src.p, src.bytes, hipMemcpyDeviceToDevice, st), "S copy");
      hipck(hipStreamSynchronize(st), "S copy");
      P.prec[p].bytes += cp.bytes;
      P.prec[p].S = cp.take();
    }
  }

  void setup(const DeviceKernel& K, const std::vector<int64_t>& xs, const std::vector<int64_t>& os_) {
    hipck(hipStreamCreate(&st), "hipStreamCreate");
    rbck(rocblas_create_handle(&bl.h), "rocblas_create_handle");
    rbck(rocblas_set_stream(bl.h, st), "rocblas_set_stream");
    bl.st = st;
    std::vector<int32_t> xn1(K.nx), xn2(K.nx), w1(K.nxi), w2(K.nxi);
    std::vector<double> c1, c2;
    if (K.kind == 1) {
      c1.resize(K.nx);
      c2.resize(K.nx);
    }
    for (int64_t i = 0; i < K.nx; ++i) {
      const double a = K.x[2 * i], b = K.x[2 * i + 1];
      if (K.kind == 0) {
        xn1[i] = (int32_t)std::llround(a);
        xn2[i] = (int32_t)std::llround(b);
      } else {
        xn1[i] = (int32_t)std::llround(a * (double)K.n);
        xn2[i] = (int32_t)std::llround(b * (double)K.n);
        c1[i] = K.c_scale * (2.0 + std::sin(2.0 * M_PI * a) * std::sin(2.0 * M_PI * b)) / 16.0;
        c2[i] = K.c_scale * (2.0 + std::cos(2.0 * M_PI * a) * std::cos(2.0 * M_PI * b)) / 16.0;
      }
    }
    for (int64_t i = 0; i < K.nxi; ++i) {
      w1[i] = (int32_t)std::llround(K.xi[2 * i]);
      w2[i] = (int32_t)std::llround(K.xi[2 * i + 1]);
    }
    d_xn1 = upload(xn1, st);
    d_xn2 = upload(xn2, st);
    d_w1 = upload(w1, st);
    d_w2 = upload(w2, st);
    if (K.kind == 1) {
      d_c1 = upload(c1, st);
      d_c2 = upload(c2, st);
    }
    ks = KSpec{K.kind, K.n, d_xn1.as<int32_t>(), d_xn2.as<int32_t>(), d_c1.as<double>(), d_c2.as<double>(),
               d_w1.as<int32_t>(), d_w2.as<int32_t>()};
    xcall.resize(xt.npts);
    ocall.resize(ot.npts);
    for (int64_t i = 0; i < xt.npts; ++i) xcall[i] = (int32_t)xs[xt.perm[i]];
    for (int64_t i = 0; i < ot.npts; ++i) ocall[i] = (int32_t)os_[ot.perm[i]];
    d_xcall = upload(xcall, st);
    d_ocall = upload(ocall, st);
    rank.assign(L + 1, {});
    pieces.assign(L, {});
  }
};

}  // namespace

Error build_part_device(const Tree& xt, const Tree& ot, const std::vector<int64_t>& xs,
                        const std::vector<int64_t>& os, const DeviceKernel& K, const mbf_opts& o,
                        uint32_t prec_mask, DevPart& P) {
  try {
    Builder b(xt, ot, o, prec_mask);
    b.setup(K, xs, os);
    g_tm = Timers();
    b.middle();
    b.log("middle level done");
    g_tm.report("middle level");
    b.u_side();
    b.log("U recursion done");
    g_tm.report("U recursion");
    b.v_side();
    b.log("V recursion done");
    g_tm.report("V recursion");
    b.mXu.release();
    b.mXv.release();
    b.assemble(os.data(), P);
    b.log("assembled");
    return {MBF_OK, ""};
  } catch (const DevErr& e) {
    return {e.st, e.what()};
  }
}

Error build_center_device(const DeviceKernel& K, const std::vector<int64_t>& idx, uint32_t prec_mask, DevFactor& F) {
  try {
    hipStream_t st = nullptr;
    hipck(hipStreamCreate(&st), "hipStreamCreate");
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{st};
    std::vector<int32_t> xn1(K.nx), xn2(K.nx), w1(K.nxi), w2(K.nxi), rows(K.nx), cols(idx.size());
    std::vector<double> c1, c2;
    if (K.kind == 1) {
      c1.resize(K.nx);
      c2.resize(K.nx);
    }
    for (int64_t i = 0; i < K.nx; ++i) {
      const double a = K.x[2 * i], b = K.x[2 * i + 1];
      if (K.kind == 0) {
        xn1[i] = (int32_t)std::llround(a);
        xn2[i] = (int32_t)std::llround(b);
      } else {
        xn1[i] = (int32_t)std::llround(a * (double)K.n);
        xn2[i] = (int32_t)std::llround(b * (double)K.n);
        c1[i] = K.c_scale * (2.0 + std::sin(2.0 * M_PI * a) * std::sin(2.0 * M_PI * b)) / 16.0;
        c2[i] = K.c_scale * (2.0 + std::cos(2.0 * M_PI * a) * std::cos(2.0 * M_PI * b)) / 16.0;
      }
      rows[i] = (int32_t)i;
    }
    for (int64_t i = 0; i < K.nxi; ++i) {
      w1[i] = (int32_t)std::llround(K.xi[2 * i]);
      w2[i] = (int32_t)std::llround(K.xi[2 * i + 1]);
    }
    for (size_t j = 0; j < idx.size(); ++j) cols[j] = (int32_t)idx[j];
    DBuf a1 = upload(xn1, st), a2 = upload(xn2, st), b1 = upload(w1, st), b2 = upload(w2, st);
    DBuf e1 = upload(c1, st), e2 = upload(c2, st), dr = upload(rows, st), dc = upload(cols, st);
    KSpec ks{K.kind, K.n, a1.as<int32_t>(), a2.as<int32_t>(), e1.as<double>(), e2.as<double>(), b1.as<int32_t>(),
             b2.as<int32_t>()};
    const int nc = (int)idx.size();
    std::vector<EntryDesc> ed = {{dr.as<int32_t>(), dc.as<int32_t>(), (int32_t)K.nx, nc}};
    DBuf d_ed = upload(ed, st);
    DBuf KC(zb((int64_t)K.nx * nc));
    hipLaunchKernelGGL(k_entries, dim3(gridx((int64_t)K.nx * nc), 1), dim3(256), 0, st, ks, d_ed.as<EntryDesc>(),
                       (int)K.nx, nc, KC.as<z2>(), (int64_t)K.nx * nc, (int64_t)1, (int64_t)K.nx, 0, 1);
    hipck(hipGetLastError(), "k_entries");
    F.n_center = nc;
    DBuf ci = upload(cols, st);
    F.d_center_idx = ci.as<int32_t>();
    ci.take();
    const int64_t n = (int64_t)K.nx * nc;
    for (int p = 0; p < kNumPrec; ++p) {
      if (!(prec_mask & (1u << p))) continue;
      PrecData& d = F.center[p];
      d.present = true;
      std::vector<PackDesc> pd = {{KC.as<z2>(), 0, (int32_t)n, (int32_t)n, 1, (int32_t)n, 0, 0, 0, 0}};
      DBuf dpd = upload(pd, st);
      DBuf out(p == MBF_C128 ? zb(n) : (size_t)n * 8);
      hipLaunchKernelGGL(k_pack, dim3(gridx(n), 1), dim3(256), 0, st, dpd.as<PackDesc>(),
                         p == MBF_C128 ? out.as<z2>() : nullptr, p == MBF_C128 ? nullptr : out.as<float2>(),
                         (ushort4*)nullptr);
      hipck(hipGetLastError(), "k_pack");
      hipck(hipStreamSynchronize(st), "center");
      d.bytes += out.bytes;
      d.center = out.take();
    }
    return {MBF_OK, ""};
  } catch (const DevErr& e) {
    return {e.st, e.what()};
  }
}

}  // namespace mbf
