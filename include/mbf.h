/*
 * mbf.h -- C ABI of libmbf: the multidimensional butterfly factorization
 * (Li, Yang, Ying, "Multidimensional Butterfly Factorization") applied on an
 * AMD MI355X (gfx950).
 *
 * The library evaluates u = K g (Section 1.1, eq. (kernel)):
 *     u(x) = sum_{xi in Omega} K(x, xi) g(xi),  x in X,
 * through the factorization of eq. (gbf):
 *     K ~ U^L G^{L-1} ... G^h M^h (H^h)^* ... (H^{L-1})^* (V^L)^*,
 * applied right to left on the GPU (Section 2.5: cost = number of nonzeros).
 * Singular kernels e^{2 pi i Phi(x, xi)} use the polar split (Section 3.2)
 * or the multiscale split K = K_C R_C + sum_t K_t R_t (Section 4.2,
 * eq. (msumd), eq. (f1)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Ordering:  row i of K (and of u) follows the caller's order of X; column j
 *            (and row j of g) follows the caller's order of Omega.  Tree
 *            permutations are internal.
 * Layout:    complex values are interleaved (re, im): complex64 = 2 floats,
 *            complex128 = 2 doubles.  RHS blocks are column-major with a
 *            leading dimension ld >= number of points.
 * Ownership: g, u, v, h and workspace are device pointers owned by the caller.
 *            A factor handle owns its device memory until mbf_destroy.
 * Streams:   `stream` is a hipStream_t passed as void* (NULL = default
 *            stream).  Apply calls only enqueue work: they never synchronize
 *            and never allocate.  A factor is immutable after build/import;
 *            concurrent applies on different streams with separate
 *            workspaces are safe.
 * Errors:    every call returns an mbf_status; no exception crosses the ABI.
 *            mbf_last_error() returns a thread-local message for the last
 *            failure on the calling thread.
 */
#ifndef MBF_H
#define MBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MBF_OK = 0,
  MBF_ERR_INVALID_ARG = -1,
  MBF_ERR_OOM = -2,
  MBF_ERR_CALLBACK = -3,
  MBF_ERR_HIP = -4,
  MBF_ERR_UNSUPPORTED = -5,
  MBF_ERR_BUSY = -6,
  MBF_ERR_IO = -7
} mbf_status;

/* Arithmetic of the apply.  A factor keeps one device copy per precision
 * requested in its precision mask (bit 1 << mbf_prec).
 *   MBF_C128      complex128 factors and vectors, FP64 arithmetic.
 *   MBF_C64       complex64 factors and vectors, FP32 arithmetic.
 *   MBF_C64_SPLIT_BF16  complex64 vectors; each stage block product runs on
 *                 BF16 matrix cores as hi*hi + hi*lo + lo*hi with FP32
 *                 accumulation (factor entry = hi + lo, both BF16).      */
typedef enum {
  MBF_C128 = 0,
  MBF_C64 = 1,
  MBF_C64_SPLIT_BF16 = 2
} mbf_prec;

typedef enum { MBF_SPLIT_NONE = 0, MBF_SPLIT_POLAR = 1, MBF_SPLIT_MULTISCALE = 2 } mbf_split;

typedef struct mbf_factor_s* mbf_factor;

/* Kernel-entry callback (build case (ii), Section 2.3: every entry of K can
 * be evaluated in O(1)).  Must write out[a + b*m] = K(x[rows[a]], xi[cols[b]])
 * as interleaved complex128 for a < m, b < k, where rows / cols index the
 * point arrays given to mbf_build.  Return 0 on success; any other value
 * aborts the build with MBF_ERR_CALLBACK.  Called concurrently from several
 * host threads. */
typedef int (*mbf_entry_cb)(void* user, int64_t m, const int64_t* rows, int64_t k,
                            const int64_t* cols, double* out);

/* Ready-made callbacks.  `user` points to an mbf_kernel_params.
 *   mbf_kernel_dft:  K = exp(-2 pi i x.xi / n), x and xi integer coordinates
 *                    (the 2D DFT; x.xi is reduced modulo n exactly).
 *   mbf_kernel_fio:  Example 1 of Section 3.3, eq. (example1phi):
 *                    K = exp(2 pi i Phi), Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2),
 *                    c1 = c_scale (2 + sin 2pi x1 sin 2pi x2)/16,
 *                    c2 = c_scale (2 + cos 2pi x1 cos 2pi x2)/16,
 *                    x = (n1/n, n2/n), xi integer.
 *   mbf_kernel_fio_points: the same kernel for arbitrary real points x and
 *                    xi (general point sets): Phi evaluated directly in
 *                    FP64, without the grids' exact reduction of x.xi
 *                    (n unused).                                         */
typedef struct {
  int64_t n;        /* grid side */
  double c_scale;   /* FIO only: 1 = Example 1, 0 = linear phase x.xi */
  const double* x;  /* X points (2 doubles each), as given to mbf_build */
  const double* xi; /* Omega points */
} mbf_kernel_params;
int mbf_kernel_dft(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                   double* out);
int mbf_kernel_fio(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                   double* out);
int mbf_kernel_fio_points(void* user, int64_t m, const int64_t* rows, int64_t k, const int64_t* cols,
                          double* out);

/* Build options.
 *   tol        block-relative truncation: keep sigma_k > tol * sigma_1
 *              (the paper fixes a rank r instead; max_rank caps it).
 *   max_rank   rank cap per block (>= 1).
 *   depth      tree depth L (both trees).  0 = automatic: uniform leaves of
 *              leaf_side x leaf_side points on a grid of side n.
 *   leaf_side  leaf side for depth = 0 (power of two dividing n).
 *   grid_n     side n of the grids (needed by the polar and multiscale maps);
 *              0 = general point sets (Section 2.6): the trees cover the
 *              bounding squares of X and Omega (Omega through the polar map
 *              with R = max |xi| for MBF_SPLIT_POLAR) to the given depth
 *              (>= 1), nodes without points are dropped; host builder only,
 *              no multiscale split.
 *   split      MBF_SPLIT_*.
 *   center_side multiscale only: side of the dense center square Omega_C
 *              (Section 4.3 uses 16).
 *   oversample random-sampling oversampling (extra rows / columns).
 *   seed       seed of the random sampling.
 *   prec_mask  bit (1 << mbf_prec) for every precision to keep on device.
 *   threads    host threads of the host builder (0 = OMP_NUM_THREADS when
 *              set, else the CPUs in the process's affinity mask).
 *   builder    MBF_BUILD_HOST: FP64 on the host, any entry callback.
 *              MBF_BUILD_DEVICE: FP64 on the current HIP device; the entries
 *              are evaluated on the device, so the callback must be one of
 *              the ready-made kernels (mbf_kernel_dft / mbf_kernel_fio) and
 *              tol >= 1e-7 (its orthonormal bases come from Gram matrices,
 *              which resolve singular values down to about 1e-8 of the
 *              largest).  Otherwise MBF_ERR_UNSUPPORTED.
 *   device_mem_gb  MBF_BUILD_DEVICE: bound on the builder's scratch memory
 *              (GiB; 0 = a third of the device memory free when each part's
 *              build starts, between 48 and 128 GiB, at most 90% of what is
 *              free).  The finished factors are not counted.               */
typedef enum { MBF_BUILD_HOST = 0, MBF_BUILD_DEVICE = 1 } mbf_builder;
typedef struct {
  double tol;
  int32_t max_rank;
  int32_t depth;
  int32_t leaf_side;
  int32_t grid_n;
  int32_t split;
  int32_t center_side;
  int32_t oversample;
  uint64_t seed;
  uint32_t prec_mask;
  int32_t threads;
  int32_t builder;
  int32_t device_mem_gb;
} mbf_opts;

/* Build a factorization from point sets and an entry callback (Section 2,
 * case (ii)): middle-level factorization by SVD via random sampling
 * (Sections 2.1, 2.3, eq. (Kij), form eq. (lowrank1)), then the recursive
 * factorizations of U^h and V^h by truncated SVD (Section 2.4, eq. (blockF),
 * form eq. (lowrank2)); polar (Section 3.2) or multiscale (Section 4.2)
 * splits per opts->split.  x: nx points, xi: nxi points, 2 doubles each
 * (host memory, read during the call only).  The build runs in FP64 on the
 * host or on the current HIP device (opts->builder); the factors are left
 * on the device in every precision of opts->prec_mask before the call
 * returns (the call synchronizes the device).  The device builder follows
 * the same steps: the random-sampling SVD of every middle-level block
 * (representative columns and rows by pivoted QR of sampled blocks,
 * orthonormal bases of the representative columns and rows, the middle
 * matrix from a sampled sub-block, its SVD), then the recursive truncated
 * SVDs of the merged blocks, level by level.  Errors: MBF_ERR_INVALID_ARG
 * (bad sizes or options), MBF_ERR_CALLBACK (callback returned nonzero;
 * nothing leaks), MBF_ERR_UNSUPPORTED (device builder with another
 * callback or tol < 1e-7), MBF_ERR_OOM, MBF_ERR_HIP. */
mbf_status mbf_build(int32_t dim, int64_t nx, const double* x, int64_t nxi, const double* xi,
                     mbf_entry_cb cb, void* user, const mbf_opts* opts, void* stream,
                     mbf_factor* out);

/* Black box of build case (i) (Section 2.3: fast products with K and K^*
 * are available).  adjoint = 0: out = K in, with in nxi x ncols and out
 * nx x ncols; adjoint = 1: out = K^* in, with in nx x ncols and out
 * nxi x ncols.  Host buffers of interleaved complex128, column-major with
 * the row count as leading dimension, valid during the call only; point
 * order as given to mbf_build_matvec.  Return 0 on success; any other
 * value aborts the build with MBF_ERR_CALLBACK.  Called from one host
 * thread at a time. */
typedef int (*mbf_matvec_cb)(void* user, int32_t adjoint, int64_t ncols, const double* in, double* out);

/* Build case (i) (Section 2.3; PBF-m of Section 3.2, MBF-m of Section 4.2):
 * the factorization of a K known only through mv.  Trees, splits and the
 * recursive factorizations of U^h and V^h are those of mbf_build; every
 * middle-level block K_{A,B} is factored by the SVD via random
 * matrix-vector products (Section 2.1, first option) from K C^P_B and
 * K^* R^P_A, where C^P_B (R^P_A) holds Gaussian entries on the points of the
 * Omega node B (X node A) and zeros elsewhere: one product with K per
 * middle-level Omega node, one with K^* per middle-level X node, all of
 * them taken before the factorization.  Bases of at most max_rank columns
 * come from pivoted QR of the products; the middle matrix
 * M = pinv(R^* Q_col) (R^* K C) pinv(Q_row^* C) from two least-squares
 * solves; its SVD truncated by tol.  The dense center of the multiscale
 * split is K applied to its unit vectors.
 *   probes  NULL: Gaussian probes drawn from opts->seed; else q =
 *           max_rank + oversample columns of C (nxi x q) followed by those
 *           of R (nx x q), interleaved complex128, column-major (host,
 *           read during the call).  oversample must be >= 1.
 * opts->builder must be MBF_BUILD_HOST (else MBF_ERR_UNSUPPORTED).  Other
 * errors as mbf_build. */
mbf_status mbf_build_matvec(int32_t dim, int64_t nx, const double* x, int64_t nxi, const double* xi,
                            mbf_matvec_cb mv, void* user, const mbf_opts* opts, const double* probes,
                            void* stream, mbf_factor* out);

/* Import an already built factorization: the factors of eq. (gbf) as host
 * arrays (FP64), read during the call only.  Used to apply factorizations
 * built elsewhere.  Trees: quadtrees of depth L whose nodes are numbered in
 * Z-order (Section 2.2, Fig. 1; child t of node i is 4i+t).  A tree is given
 * by the Morton code of the leaf holding each point; nodes without points
 * are absent, and the points of a leaf are ordered by increasing index.
 * Stage s (0..L) pairs: (A at level s of T_X, B at level L-s of T_Omega),
 * enumerated A-major, B-minor, over nonempty nodes in increasing Morton
 * code.  h = floor(L/2).  All matrices are column-major complex128.
 *   ranks     for s = 0..L, one int32 per stage-s pair (concatenated).
 *   v_leaf    (V^L)^* blocks: for every nonempty Omega leaf B, V_B of size
 *             |B| x rank_0(root, B) (y_B = V_B^* g_B).
 *   h_blocks  for s = 0..h-1, for every A at X-level s, for every B' at
 *             Omega-level L-s-1, for every nonempty child B of B' in order:
 *             H_{B,A} of size rank_s(A,B) x sum_t rank_{s+1}(child_t A, B')
 *             (columns grouped by the children of A in order); the stage
 *             product is y_{(child_t A, B')} = sum_B H_{B,A}[:, t-group]^* y_{(A,B)}
 *             (Section 2.4.2, mirror of eq. (blockF)).
 *   s_mid     for every stage-h pair in pair order, rank_h values of
 *             S = Sigma^{-1} (eq. (lowrank1), eq. (Kij)); M^h applies them.
 *   g_blocks  for s = h..L-1, for every A at X-level s, for every B' at
 *             Omega-level L-s-1, for every child A_t of A in order:
 *             G_{A_t,B'} of size rank_{s+1}(A_t,B') x sum_sigma rank_s(A, child_sigma B')
 *             (eq. (blockF), eq. (RSh2)).
 *   u_leaf    for every X leaf A: U_A of size |A| x rank_L(A, root).
 * Errors: MBF_ERR_INVALID_ARG when sizes are inconsistent. */
typedef struct {
  int32_t depth;                 /* L */
  int64_t nx, nxi;               /* points of X and of Omega */
  const int64_t* x_leaf_code;    /* nx Morton codes at level L */
  const int64_t* xi_leaf_code;   /* nxi Morton codes at level L */
  const int32_t* ranks;
  const double* v_leaf;
  const double* h_blocks;
  const double* s_mid;
  const double* g_blocks;
  const double* u_leaf;
} mbf_import_desc;

mbf_status mbf_import(const mbf_import_desc* d, uint32_t prec_mask, void* stream, mbf_factor* out);

/* Multiscale assembly (Section 4.2, eq. (f1)): K ~ K_C R_C + sum_t K_t R_t.
 * parts[t] is a factorization of K restricted to X x Omega_t, and
 * part_idx[t] (part_n[t] entries) lists, in that factorization's column
 * order, the Omega indices of Omega_t.  center holds K_C as a dense
 * column-major complex128 nx x n_center matrix on the host, center_idx its
 * Omega indices.  The new handle takes ownership of the parts (do not
 * destroy them separately, also on failure). */
mbf_status mbf_multiscale_assemble(int32_t nparts, mbf_factor* parts, const int64_t* const* part_idx,
                                   const int64_t* part_n, int64_t nxi, int64_t n_center,
                                   const int64_t* center_idx, const double* center,
                                   uint32_t prec_mask, void* stream, mbf_factor* out);

/* Checkpoint / resume of built factorizations.  mbf_save writes the
 * precisions in prec_mask (0 = every precision the handle holds) to a
 * versioned binary file (device -> host in chunks; synchronous).  mbf_load reads it back onto the current device,
 * keeping the precisions in prec_mask (0 = all stored).  Errors: MBF_ERR_IO
 * (cannot open, write failure, wrong magic / version, corrupted or
 * truncated file: nothing is left allocated), MBF_ERR_UNSUPPORTED (a
 * requested precision is not in the file), MBF_ERR_OOM. */
mbf_status mbf_save(mbf_factor f, uint32_t prec_mask, const char* path);
mbf_status mbf_load(const char* path, uint32_t prec_mask, void* stream, mbf_factor* out);

/* Bytes of device workspace needed by an apply of nrhs columns. */
mbf_status mbf_workspace_size(mbf_factor f, mbf_prec p, int64_t nrhs, size_t* bytes);

/* u = K g.  g: nxi x nrhs (ld ldg), u: nx x nrhs (ld ldu), device memory of
 * the precision's vector type (complex128 for MBF_C128, complex64
 * otherwise).  Overwrites u.  Errors: MBF_ERR_INVALID_ARG (null pointer,
 * ld too small, workspace too small), MBF_ERR_UNSUPPORTED (precision not in
 * the factor's mask), MBF_ERR_HIP (launch failure).
 * Multiscale factorizations (eq. (f1)): with a workspace of
 * mbf_workspace_size bytes, the coronas' parts and the dense center run on
 * side streams of `stream` (created on the first call with that stream and
 * device, kept until the process ends), ordered after the work already on
 * `stream` and joined back into it before the call returns; the sums are
 * added into u in the same order as one after the other, so results do not
 * depend on it.  While `stream` is being captured into a graph, or with
 * MBF_PART_STREAMS=0, or with a workspace that only holds the parts one after
 * the other, everything runs on `stream`.  Calls on one stream must come
 * from one host thread at a time. */
mbf_status mbf_apply(mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg, void* u,
                     int64_t ldu, void* workspace, size_t ws_bytes, void* stream);

/* u = K g without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels as mbf_apply, with the workspace taken
 * from a fixed device array of the library (mbf_scratch_bytes() bytes,
 * 128 MiB; one copy per device, held until the process ends) instead of the
 * caller's workspace.  Arguments as for mbf_apply.  Errors as mbf_apply,
 * plus MBF_ERR_INVALID_ARG when the apply needs more workspace than the
 * scratch holds (use mbf_apply then).  A multiscale factorization's parts
 * run one after the other on `stream` here (no side streams), which needs
 * at most mbf_workspace_size(f, p, nrhs) bytes, less when the parts would
 * otherwise run side by side.  The first call on a device looks up the scratch's
 * address there.  All calls on one device share its scratch: calls that
 * overlap on one device (concurrent streams or threads) race and must be
 * serialized by the caller. */
mbf_status mbf_apply_scratch(mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg, void* u,
                             int64_t ldu, void* stream);
size_t mbf_scratch_bytes(void);

/* v = K^* h: the chain of eq. (gbf) in reverse order with every factor
 * conjugate-transposed.  h: nx x nrhs (ld ldh), v: nxi x nrhs (ld ldv).
 * Streams, workspace and errors as mbf_apply (the multiscale parts write
 * disjoint entries of v). */
mbf_status mbf_apply_adjoint(mbf_factor f, mbf_prec p, int64_t nrhs, const void* h, int64_t ldh,
                             void* v, int64_t ldv, void* workspace, size_t ws_bytes, void* stream);

/* Sizes of a factorization (Section 2.5, Table 1: apply cost = nnz). */
typedef struct {
  int32_t depth;          /* L (0 for multiscale handles) */
  int32_t mid;            /* h */
  int32_t nparts;         /* 1, or the number of coronas */
  int32_t max_rank[33];   /* per stage s = 0..L: max pair rank (first part) */
  int64_t nx, nxi;
  int64_t nnz;            /* complex nonzeros of all factors (incl. dense center) */
  int64_t nnz_stage_max;  /* largest single-stage block nonzeros */
  int64_t state_rows_max; /* largest stage state (rows) */
  uint32_t prec_mask;
  size_t device_bytes;    /* factor bytes resident on the device */
} mbf_info_t;
mbf_status mbf_info(mbf_factor f, mbf_info_t* out);

/* Autotuner of the stage kernels: for every stage shape of f at this
 * precision and RHS count, times each stage-kernel variant (reduction chunk
 * 16 / 32 complex entries, register prefetch off / on) on scratch data in
 * `workspace` (overwritten; same size as for mbf_apply), forward and
 * adjoint, and keeps the fastest for all later applies of that shape in
 * this process.  When the environment variable MBF_TUNE_FILE names a file,
 * choices are appended to it and read back by later processes.  Waits for
 * its own launches (synchronizes `stream`).  *tuned = stage shapes timed.
 * Applies without tuning use a fixed default variant. */
mbf_status mbf_autotune(mbf_factor f, mbf_prec p, int64_t nrhs, void* workspace, size_t ws_bytes, void* stream,
                        int32_t* tuned);

/* Per-launch timing of the apply kernels with HIP events (instrumentation,
 * Section 2.5: cost per factor).  mbf_profile_begin creates 2 * max_launches
 * events (it may allocate; call it outside graph capture and timed loops).
 * While active, every kernel that mbf_apply / mbf_apply_adjoint enqueues
 * records an event pair on its stream, until max_launches are used.
 * mbf_profile_end waits for those events, writes up to `cap` records and
 * the number of records to *count, and stops profiling.
 *   kind:  0 leaf project, 1 stage block product, 2 leaf reconstruct,
 *          3 dense center (multiscale)
 *   flops: algorithmic real flops of the launch (8 per complex multiply-add
 *          of a factor entry with one vector entry)
 *   bytes: algorithmic HBM bytes (factor entries read once + vectors read
 *          and written once) */
typedef struct {
  int32_t kind;
  int32_t part;
  int32_t stage;
  int32_t prec;
  double ms;
  double flops;
  double bytes;
} mbf_launch_record;
mbf_status mbf_profile_begin(mbf_factor f, int32_t max_launches);
mbf_status mbf_profile_end(mbf_factor f, mbf_launch_record* out, int32_t cap, int32_t* count);

/* Serving: a request loop over resident factorizations with continuous
 * batching and memory admission (no passage of the paper: the batched,
 * served form of eq. (gbf)'s apply).  mbf_server_create reserves
 * mem_budget bytes of device memory (the only allocation of the server) and
 * nslots HIP streams (default priority).  A dispatcher thread forms batches
 * from queued requests on the same (factor, precision), up to max_batch_rhs
 * columns; a batch is admitted when a slot is free and the pool can hold its
 * staging (g and u blocks) and workspace; batches on different slots run
 * concurrently.  Requests that arrive while others are on the GPU join the
 * next batches as slots and memory free up.  When several queued requests
 * together exceed the pool, the later ones wait for a following batch; only
 * a request that cannot fit the whole budget on its own fails.
 * flags: 0, or MBF_SERVER_GRAPHS: each slot keeps one fixed region of the
 * pool for its staging blocks and workspace (sized for the largest batch it
 * has run; grown on demand, and the regions of idle slots are given back
 * when the pool cannot otherwise hold a growth), and runs each batch's apply
 * as one launch of a HIP graph captured once per (factor, precision, batch
 * width) on the slot's stream; batch widths are rounded up to a power of two
 * of at least 16 columns, within max_batch_rhs (the padding columns compute
 * results that are never read).  Without it every batch enqueues the apply's
 * kernels one by one into a reservation of its own.  Results are the same.
 *   submit: u = K g for one request (device pointers owned by the caller,
 *           unchanged until the request completes); returns its id.
 *           Readiness: the server's streams do not follow the caller's
 *           streams.  If g is produced by device work that may still be
 *           running, pass an event recorded after that work as ready_event
 *           (hipEvent_t as void*; it must stay valid until the request
 *           completes): the batch waits for it before reading g.  With
 *           ready_event = NULL, g must already be complete on the device.
 *   poll:   *done = 1 once u holds the result, and the request's record is
 *           then released; latency = completion - submission on the host
 *           clock (microseconds).  A request that failed reports *done = 1
 *           and returns its error: MBF_ERR_OOM when it can never fit the
 *           budget, MBF_ERR_HIP when its batch could not be enqueued or
 *           failed on the device (u is then undefined).  An id that was never
 *           issued or whose completion was already reported returns
 *           MBF_ERR_INVALID_ARG.  At most 2^20 unpolled records are kept (the
 *           oldest are dropped beyond that).
 *   drain:  waits until every submitted request has completed; returns
 *           MBF_ERR_HIP if any batch failed since the server was created.
 *   stats:  p50 / p99 / mean latency over the last 2^20 successful requests,
 *           requests, RHS, batches, the largest number of batches in flight
 *           at once, graphs captured and batches run as a graph launch, wall
 *           time first submit -> last completion.
 * A factor must outlive every request that names it.  Submit, poll, drain
 * and stats may be called from any host thread. */
typedef struct mbf_server_s* mbf_server;
typedef struct {
  int64_t requests, rhs, batches, max_concurrent_batches, graphs_captured, graph_batches;
  double p50_us, p99_us, mean_us, wall_s;
} mbf_server_stats_t;
#define MBF_SERVER_GRAPHS 1u
mbf_status mbf_server_create(size_t mem_budget, int32_t nslots, int64_t max_batch_rhs, uint32_t flags,
                             mbf_server* out);
mbf_status mbf_server_submit(mbf_server s, mbf_factor f, mbf_prec p, int64_t nrhs, const void* g, int64_t ldg,
                             void* u, int64_t ldu, void* ready_event, uint64_t* id);
mbf_status mbf_server_poll(mbf_server s, uint64_t id, int32_t* done, double* latency_us);
mbf_status mbf_server_drain(mbf_server s);
mbf_status mbf_server_stats(mbf_server s, mbf_server_stats_t* out);
void mbf_server_destroy(mbf_server s);

void mbf_destroy(mbf_factor f);
const char* mbf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBF_H */
