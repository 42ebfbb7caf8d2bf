// Internal data structures of libmbf (host side).
//
// A factorization (eq. (gbf)) is held as
//   * two quadtrees (Section 2.2) over X and over Omega (or over the polar
//     image P, Section 3.2, or over a corona's bounding square, Section 4.2);
//   * per stage s = 0..L the ranks of all pairs (A at X-level s,
//     B at Omega-level L-s), A-major / B-minor over nonempty nodes;
//   * the leaf factors V^L (Omega leaves) and U^L (X leaves);
//   * per stage s = 0..L-1 one dense "block" per (A at X-level s,
//     B' at Omega-level L-s-1): the matrix that maps the vectors of the
//     pairs (A, child_sigma B') to those of (child_tau A, B').  For s < h it
//     gathers the blocks H_{child_sigma B', A}^* (Section 2.4.2), for s >= h
//     the blocks G_{child_tau A, B'} (Section 2.4.1, eq. (blockF));
//   * the middle scaling S = Sigma^{-1} of M^h (eq. (lowrank1), eq. (Kij)).
#pragma once

#include <complex>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mbf.h"

namespace mbf {

using cd = std::complex<double>;

struct Tree {
  int L = 0;
  int64_t npts = 0;
  std::vector<std::vector<int64_t>> code;    // [l] Morton codes of nonempty nodes, ascending
  std::vector<std::vector<int64_t>> off;     // [l] nn+1 offsets into perm
  std::vector<std::vector<int32_t>> cfirst;  // [l<L] nn+1 child ranges (indices at level l+1)
  std::vector<int64_t> perm;                 // tree order -> point index (leaf-major, index-ascending)
  int32_t nn(int l) const { return (int32_t)code[l].size(); }
  int64_t size(int l, int32_t i) const { return off[l][i + 1] - off[l][i]; }
};

// Build a tree from the Morton code of the leaf (level L) holding each point.
Tree tree_from_leaf_codes(int L, int64_t npts, const int64_t* leaf_code);
// Morton code with the first coordinate as the more significant bit (Fig. 1).
int64_t morton2(int64_t c1, int64_t c2, int level);

struct HostFactor {
  int L = 0, m = 0;
  Tree xt, ot;
  std::vector<std::vector<int32_t>> rank;      // [s] nX(s) * nO(L-s)
  std::vector<std::vector<cd>> V0;             // [Omega leaf] |B| x r, column-major
  std::vector<std::vector<cd>> UL;             // [X leaf]     |A| x r, column-major
  std::vector<double> S;                       // stage-h rows, in state order
  std::vector<std::vector<cd>> W;              // [s] blocks concatenated, each M x K column-major
  std::vector<std::vector<int64_t>> Woff;      // [s] nblk+1 element offsets
  // Dense center (multiscale only): nx x nc column-major, and its Omega indices.
  std::vector<cd> center;
  std::vector<int64_t> center_idx;

  int64_t pair(int s, int32_t ia, int32_t ib) const {
    return (int64_t)ia * ot.nn(L - s) + ib;
  }
};

// Assemble the stage blocks W from the paper's H / G blocks.  Inputs are
// given in the import order documented in mbf.h.
void assemble_blocks(HostFactor& f, const double* h_blocks, const double* g_blocks);

// Number of complex nonzeros (Section 2.5).
int64_t host_nnz(const HostFactor& f);

// Thread-local error reporting.
void set_error(const std::string& s);
struct Error {
  mbf_status st;
  std::string msg;
};

}  // namespace mbf
