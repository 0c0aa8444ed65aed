/*
 * tnrsvd.h -- C ABI of the MI355X (gfx950) Tensor Network randomized SVD.
 *
 * Method: Batselier, Yu, Daniel, Wong, "Computing low-rank approximations of
 * large-scale matrices with the Tensor Network randomized SVD" (arXiv
 * 1707.07803): the randomized SVD of Algorithm 5.1 carried out entirely in
 * MPO form (Sec. 5), with the subspace iteration of Algorithm 5.4, the MPO
 * products of Sec. 5.2, the thin QR / economical SVD sweeps of Algorithms 5.2
 * and 5.3, and the SVD-based rounding of Sec. 3 fused into those sweeps.
 *
 * Orientation.  The paper carries the K columns of the random MPO, of Y and
 * of Q on the FIRST core and sweeps right-to-left.  This library uses the
 * mirror image: the K leg rides on the LAST core and the orthogonalisation
 * sweeps run left-to-right.  Singular values are identical; singular vectors
 * are those of the matrix with the same (little-endian, eq. (1)) row and
 * column multi-indices.
 *
 * Layouts (all C order, 0-based, little-endian multi-indices as in eq. (1)):
 *   A core i       (R_i, I_i, J_i, R_{i+1}),  R_0 = R_d = 1 (i = 0..d-1)
 *   basis core i   (r_i, n_i, r_{i+1}); the last core is (r_{d-1}, n_{d-1}, K)
 *                  where n = I (row space: Q, U) or n = J (column space: V)
 *   product rank   p = a * r + c  (a: A rank index, c: basis rank index)
 *
 * Precision.  Contractions run in the precision chosen in tnrsvd_opts
 * (FP64; FP32 with FP32 accumulation; or BF16 storage of A, the basis and
 * the products with FP32 accumulation); every QR, SVD and rank decision of
 * the sweeps runs in FP64.  A BF16 solve can be refined by one FP32 power
 * step (tnrsvd_refine).
 *
 * Threading.  A handle is bound to one HIP device and one stream (borrowed,
 * never synchronised except where noted).  Calls on one handle must not
 * overlap; different handles are independent.  No call throws across the
 * ABI; every entry point returns a tnrsvd_status and records a message that
 * tnrsvd_last_error() returns (thread local).
 */
#ifndef TNRSVD_H
#define TNRSVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tnrsvd_s* tnrsvd_t;
typedef struct tnrsvd_rounded_s* tnrsvd_rounded_t;

typedef enum {
  TNRSVD_OK = 0,
  TNRSVD_E_INVALID = -1,   /* null pointer, bad enum, bad option value      */
  TNRSVD_E_SHAPE = -2,     /* rank/dimension mismatch, K larger than prod I */
                           /* or prod J, capacity exceeded                  */
  TNRSVD_E_STATE = -3,     /* call out of the order of Algorithm 5.4        */
  TNRSVD_E_NOMEM = -4,     /* device allocation failed (nothing leaked)     */
  TNRSVD_E_DEVICE = -5,    /* HIP runtime error                             */
  TNRSVD_E_NONFINITE = -6  /* NaN/Inf in an input core (only if checked)    */
} tnrsvd_status;

typedef enum {
  TNRSVD_F64 = 0,          /* FP64 contractions                              */
  TNRSVD_F32 = 1,          /* FP32 contractions, FP32 accumulation           */
  TNRSVD_BF16 = 2          /* BF16 storage (round to nearest even), FP32 acc */
} tnrsvd_precision;

/* One MPO matrix A of size (prod I) x (prod J) (Sec. 3). */
typedef struct {
  int d;                     /* number of cores, >= 1                        */
  const int64_t* rank;       /* d+1 MPO ranks, rank[0] = rank[d] = 1         */
  const int64_t* rows;       /* I_0 .. I_{d-1}                               */
  const int64_t* cols;       /* J_0 .. J_{d-1}                               */
  const void* const* core;   /* d DEVICE pointers, C-contiguous (R,I,J,R')   */
  int dtype;                 /* TNRSVD_F64 (double) or TNRSVD_F32 (float)    */
} tnrsvd_mpo;

typedef struct {
  int k;                     /* number of singular triplets returned, >= 1   */
  int p;                     /* oversampling, >= 0; K = k + p                */
  int q;                     /* power iterations used by tnrsvd_run          */
  uint64_t seed;             /* seed of the counter-based random MPO         */
  int precision;             /* tnrsvd_precision                             */
  double round_tol;          /* rounding tolerance eps >= 0 (0: none)        */
  int64_t max_rank;          /* rounding rank cap r_max (0: none)            */
  int check_finite;          /* nonzero: scan input cores for NaN/Inf        */
  void* stream;              /* hipStream_t, borrowed; NULL = null stream    */
  int orientation;           /* tnrsvd_orientation                           */
  int sketch_rank;           /* 0: off; ell in [1, 256]: sketched product    */
                             /* truncation before each ROUND (see below)     */
} tnrsvd_opts;

/*
 * Sketched product truncation (opts.sketch_rank = ell > 0; not in the paper,
 * a cheaper alternative to rounding the full product).  After every product
 * (Y = A Omega, A^T Q, A Q, the projection) whose bond ranks P_k = R_k r_k
 * exceed ell somewhere, the product is compressed to bond ranks <= ell by
 * randomize-then-orthogonalize (Al Daas, Ballard et al., SIAM J. Sci.
 * Comput. 2023): a Gaussian chain with bond ranks min(ell, P_k) sketches the
 * right parts, then a left-to-right pass keeps the Householder Q of each
 * sketched panel.  The SVD-based ROUND then runs on the compressed product,
 * whose panels are ell / r times narrower.  The sketch of the t-th product of
 * a solve (t = 0 for A Omega) for MPO b uses the Omega stream of seed + b at
 * counters from (t + 1) 2^40 on.  Exact when ell reaches the product's true
 * ranks; otherwise the error is the sketch's (small when ell exceeds the
 * ranks ROUND keeps by a margin).  Workspace: about (d - 1) P ell + 4 ell n
 * max(P, ell) doubles per MPO, allocated by tnrsvd_create.
 */

/*
 * Orientation of the K leg (the paper's Sec. 5: Omega, Y and Q carry their K
 * columns on the FIRST core and the sweeps run right to left).
 *   TNRSVD_K_LAST  (0): the library's own layout, K on the last core.
 *   TNRSVD_K_FIRST (1): the paper's layout.  The MPO is read in reversed core
 *     order with each core's rank legs swapped (the same matrix with row and
 *     column digits reversed, so the same singular values), solved in the
 *     library's layout, and every result is returned reversed back:
 *     tnrsvd_copy_factor writes core k of the paper's layout (the K leg on
 *     core 0, shape (K, n, r) there), tnrsvd_get_ranks lists the bonds from
 *     the first core, tnrsvd_backward takes dcores in the caller's order.
 *     The leading cores are merged until I_1, J_1 >= K (as in Sec. 6.3).
 *     tnrsvd_get_factor reports the paper-layout shape with *dev_ptr = NULL
 *     (the core exists only in the library's layout); tnrsvd_get_omega /
 *     tnrsvd_set_omega and tnrsvd_get_product_ranks keep the library's order.
 */
typedef enum {
  TNRSVD_K_LAST = 0,
  TNRSVD_K_FIRST = 1
} tnrsvd_orientation;

/*
 * tnrsvd_create -- validate, plan and stage `batch` independent MPOs.
 *
 * For each MPO the smallest number m of trailing cores whose row and column
 * products both reach K = k + p is contracted into one core on the device
 * (the paper merges the leading cores so that the K-core satisfies
 * K <= J (random-MPO lemma, Sec. 5.1), I >= K (Algorithm 5.2) and J >= K
 * (Algorithm 5.3); Sec. 6.3 merges 5 and 7 cores).  Cores are copied into a
 * library-owned device slab in the contraction precision, so the caller may
 * free its buffers once this call returns.  The random MPO Omega (rank 1:
 * one Gaussian vector per core and a J x K Gaussian matrix on the merged
 * core, Sec. 5.1) is drawn on the device from the counter-based SplitMix64 +
 * Box-Muller stream seeded by opts->seed; MPO b uses seed + b.
 *
 * Ownership: *out receives a handle that must be released by
 * tnrsvd_destroy.  The call synchronises the stream once (planning reads no
 * device data, but the staging copies must finish before return).
 * Errors: E_INVALID (nulls, k < 1, p < 0, q < 0, bad precision/dtype,
 * negative tolerance), E_SHAPE (rank[0] or rank[d] != 1, non-positive
 * dimension, prod I < K or prod J < K), E_NONFINITE (check_finite set and a
 * core holds NaN/Inf), E_NOMEM, E_DEVICE.
 */
tnrsvd_status tnrsvd_create(tnrsvd_t* out, int batch, const tnrsvd_mpo* mpos,
                            const tnrsvd_opts* opts);

/*
 * tnrsvd_mult -- one MPO product of Sec. 5.2 for every MPO of the handle.
 *   op 0: Y = A X, where X is Omega on the first call and afterwards the
 *         column-space basis produced by the last tnrsvd_orthogonalize;
 *   op 1: Z = A^T Q, where Q is the row-space basis of the last
 *         tnrsvd_orthogonalize.
 * Per core, the product sums over the shared mode index; ranks multiply
 * (R_i r_i).  Enqueued on the stream, no synchronisation.
 * Errors: E_INVALID (op not 0/1), E_STATE (a product is already pending, or
 * the current basis lives in the wrong space).
 */
tnrsvd_status tnrsvd_mult(tnrsvd_t h, int op);

/*
 * tnrsvd_orthogonalize -- ROUND + thin QR of the pending product
 * (Algorithm 5.2 fused with the rounding of Sec. 3 as described in Sec. 5.4,
 * mirrored): a right-to-left LQ sweep, then a left-to-right truncated-SVD
 * sweep (tolerance eps ||Y||_F / sqrt(d-1) per bond, cap r_max, the K leg
 * never truncated, rank decisions in FP64), ending in an FP64 Householder QR
 * of the last core with diag(R) >= 0.  The result becomes the current basis
 * (left-orthonormal cores).  Enqueued on the stream.
 * Errors: E_STATE (no pending product).
 */
tnrsvd_status tnrsvd_orthogonalize(tnrsvd_t h);

/*
 * tnrsvd_project -- B^T = A^T Q (B = Q^T A of Algorithm 5.1) with the
 * current row-space basis Q.  Enqueued on the stream.
 * Errors: E_STATE (no row-space basis, or a product is pending).
 */
tnrsvd_status tnrsvd_project(tnrsvd_t h);

/*
 * tnrsvd_solve -- economical SVD of B in MPO form (Algorithm 5.3 fused with
 * the rounding, mirrored): ROUND and sweep B^T to its last core, FP64
 * one-sided Jacobi SVD of that core giving sigma (descending), W (K x K) and
 * V; then U = Q W on the last core of Q (Sec. 5.4).  Keeps the first k.
 * sigma: HOST buffer of batch*k doubles (MPO b at sigma + b*k) or NULL; when
 * non-NULL the call synchronises the stream to copy it out.
 * Errors: E_STATE (tnrsvd_project has not run).
 */
tnrsvd_status tnrsvd_solve(tnrsvd_t h, double* sigma);

/*
 * tnrsvd_run -- the whole sequence: mult(0), orthogonalize,
 * q x {mult(1), orthogonalize, mult(0), orthogonalize}, project, solve
 * (Algorithm 5.4 then Algorithm 5.1).  May be called again on the same
 * handle; every call restarts from Omega.  sigma as in tnrsvd_solve.
 */
tnrsvd_status tnrsvd_run(tnrsvd_t h, double* sigma);

/*
 * tnrsvd_run_graph -- the same sequence as tnrsvd_run, captured once into a
 * HIP graph and replayed on every later call (batched solves as one graph
 * launch; not part of the paper).  The first call synchronises the handle's
 * stream and records the launch sequence on a private stream of default
 * priority; every call (the first included) replays the graph there, ordered
 * after the work already queued on the handle's stream and before any work
 * queued on it afterwards.  The graph reads Omega from the handle, so
 * tnrsvd_set_omega between calls takes effect.  No call allocates after the
 * first.  Kernel arguments are fixed at capture (device slab pointers, op,
 * tolerance, rank cap), which never change for a handle.
 * sigma as in tnrsvd_solve.  Results (factors, ranks) are those of tnrsvd_run.
 * Errors: E_STATE while profiling is on (event records cannot be captured);
 * E_DEVICE if capture or instantiation fails.
 */
tnrsvd_status tnrsvd_run_graph(tnrsvd_t h, double* sigma);

/*
 * tnrsvd_refine -- after a BF16 solve (tnrsvd_run, tnrsvd_run_graph or
 * tnrsvd_solve on a handle created with TNRSVD_BF16): one FP32 power step
 * from the BF16 basis Q -- Z = A^T Q, orthogonalize, Y = A Q_Z,
 * orthogonalize -- then an FP32 projection and solve (the randomized
 * subspace iteration of Algorithm 5.4 continued in FP32; refining a BF16
 * result is not part of the paper).  A is used in FP32, as staged by
 * tnrsvd_create before narrowing it to BF16.  Results (sigma, U, V, ranks,
 * the basis, now FP32) replace those of the BF16 solve; the next
 * tnrsvd_run or tnrsvd_run_graph starts again in BF16.
 * round_tol: the rounding tolerance of the FP32 step (the handle's own
 * tolerance, chosen above BF16 noise, is restored afterwards); the rank cap
 * is the handle's.  sigma as in tnrsvd_solve.
 * Errors: E_INVALID (round_tol negative or not finite); E_STATE (not a BF16
 * handle, no BF16 solve, or already refined).
 */
tnrsvd_status tnrsvd_refine(tnrsvd_t h, double round_tol, double* sigma);

/*
 * tnrsvd_backward -- gradient of L = sum_{j<k} dsigma_j sigma_j of the last
 * solve with respect to the ORIGINAL (unmerged) cores of every MPO: the
 * derivative of the whole pipeline of Algorithm 5.4 as run (the product Y = A
 * Omega, the rounding and orthogonalisation after every product with its
 * ranks frozen at the values the solve chose, the q power steps, the
 * projection B^T = A^T Q and the SVD of its last core, Sec. 5.4), with Omega
 * held fixed, followed by the adjoint of the trailing-core merge of
 * tnrsvd_create.  Differentiation is not part of the paper.  The products and
 * roundings are computed again here in FP64 from the staged cores and Omega
 * (nothing but the ranks is kept from the solve); each rounding is
 * differentiated in its Gram form (right Grams of the product, eigenvectors
 * of M G M^T for the kept left vectors), which computes the same map as the
 * QR/SVD sweep of Sec. 3 while staying differentiable on products of lower
 * rank than their bonds.  Valid where the kept eigenvalues of every rounding
 * are distinct and separated from the discarded ones, and the last panel of
 * every orthogonalisation has full column rank.
 * The last solve must be tnrsvd_run or tnrsvd_run_graph (or the same steps
 * one by one), not followed by tnrsvd_refine.
 * dsigma: HOST array of batch*k doubles, or NULL for all ones.
 * dcores: DEVICE pointers, one per original core (MPO 0's cores in order,
 *   then MPO 1's, ...); each receives the R x I x J x R' gradient, C order,
 *   in the dtype that MPO's cores had in tnrsvd_create.
 * Allocates its workspace per call; synchronises the stream.
 * Errors: E_INVALID (dcores NULL); E_STATE (no solve yet, or the last solve
 * was not a plain Algorithm 5.4 sequence); E_NOMEM; E_SHAPE (a last panel
 * with fewer rows than K).
 */
tnrsvd_status tnrsvd_backward(tnrsvd_t h, const double* dsigma, void* const* dcores);

/*
 * tnrsvd_backward_frozen -- the gradient of sum_{j<k} dsigma_j u_j^T A v_j with
 * the singular vectors (u_j, v_j) of the last solve held FIXED, i.e.
 * sum_j dsigma_j u_j v_j^T written into each original core by left and right
 * environments of U, A and V and the merge adjoint.  It equals
 * tnrsvd_backward where the computed subspace is exact (rank(A) <= K, nothing
 * truncated) and is much cheaper; elsewhere it is only the fixed-vector part.
 * Arguments, ownership and errors as tnrsvd_backward; the first call
 * allocates the workspace.
 */
tnrsvd_status tnrsvd_backward_frozen(tnrsvd_t h, const double* dsigma, void* const* dcores);

/*
 * tnrsvd_autotune -- choose the launch shape of the MPO x MPS contraction
 * (threads per block in {64, 128, 256, 512}, blocks per core capped at
 * {64, 256, 1024, 4096}) for each product direction by timing `reps` launches
 * of every shape on this handle's own shapes and planned ranks (batching
 * support; not part of the paper).  Runs one solve first to obtain a basis of
 * realistic ranks; afterwards every result of the handle is invalid (the
 * next call must be tnrsvd_run, tnrsvd_run_graph or tnrsvd_mult(0)), and a
 * captured graph is dropped and recaptured on the next tnrsvd_run_graph.
 * choice: NULL or 4 ints receiving (threads, cap) for Y = A X, then for
 * Z = A^T X.  Every shape computes each output with the same arithmetic, so
 * results do not depend on the choice.
 * Errors: E_INVALID (reps < 1); E_STATE (profiling on); E_DEVICE.
 */
tnrsvd_status tnrsvd_autotune(tnrsvd_t h, int reps, int* choice);

/*
 * tnrsvd_autotune_sweeps -- choose how the rounding sweeps (Sec. 3 rounding,
 * Algorithms 5.2 and 5.3 as used in Sec. 5.4) are launched on this handle by
 * timing whole solves (tnrsvd_run: one warm-up, then `reps` timed) under each
 * candidate and keeping the fastest (batching support; not part of the
 * paper).  A choice is a pair {wmin, lpt}:
 *   wmin  the fewest product columns (P) that send an MPO's right-to-left
 *         pass to the multi-workgroup launches: 129 (every panel wider than
 *         the one-workgroup register path), 257, 513, or 0 (never: the
 *         one-workgroup blocked path takes every panel); 513 and 0 are tried
 *         only when no product can exceed 512 columns (the one-workgroup
 *         path is far slower beyond), and only 0 when no product can exceed
 *         the register path; a last core of at most 256 columns never sends
 *         its MPO there (its blocked QR stays on the one-workgroup path);
 *   lpt   1: the one-workgroup sweeps dispatch the MPOs costliest first
 *         (sum over cores of n P^2), 0: in batch order; with one MPO only 1.
 * Every choice computes the same factorisations (the paths differ only in
 * the order of floating-point sums).  Afterwards the results of the handle
 * are invalid as after tnrsvd_autotune, and a captured graph is recaptured
 * on the next tnrsvd_run_graph.
 * choice: NULL or 2 ints receiving {wmin, lpt}.  The call synchronises.
 * Errors: E_INVALID (reps < 1); E_STATE (profiling on); those of tnrsvd_run.
 */
tnrsvd_status tnrsvd_autotune_sweeps(tnrsvd_t h, int reps, int* choice);

/*
 * tnrsvd_set_sweep_config -- apply a choice {wmin, lpt} of
 * tnrsvd_autotune_sweeps without timing (e.g. one kept in a cache keyed by
 * the shapes, precision and device).  choice: HOST array of 2 ints, wmin 0
 * or > 128, lpt 0 or 1.  Results of the handle become invalid as after
 * tnrsvd_autotune.  The default is {129, 1}.
 * Errors: E_INVALID (NULL or out-of-range choice).
 */
tnrsvd_status tnrsvd_set_sweep_config(tnrsvd_t h, const int* choice);

/*
 * tnrsvd_get_factor -- borrow a device pointer to one core of a result.
 *   which 0: U (row space, last core (r, I, K)), available after solve;
 *   which 1: V (column space, last core (s, J, K)), after solve; U and V
 *            keep all K singular vectors of the projected core, the first
 *            k columns belonging to the returned sigma_1..sigma_k;
 *   which 2: the current basis (Q after an orthogonalize; last core (r,n,K));
 *   which 3: the first product Y = A Omega of the last run (last (R,I,K)),
 *            valid until the next tnrsvd_mult.
 * shape receives (r, n, r', 1) and *dtype (a tnrsvd_precision code): U and
 * V are FP64, the basis and Y are stored in the contraction type (BF16 in
 * the BF16 mode; the basis is FP32 after tnrsvd_refine).  The pointer stays valid until the next call
 * on the handle other than a getter.  The call synchronises the stream
 * (ranks are read from the device).
 * Errors: E_INVALID (b, which or core out of range), E_STATE (not available).
 */
tnrsvd_status tnrsvd_get_factor(tnrsvd_t h, int b, int which, int core,
                                const void** dev_ptr, int64_t shape[4], int* dtype);

/*
 * tnrsvd_copy_factor -- copy one core described by tnrsvd_get_factor into a
 * caller-owned DEVICE buffer dst (shape[0]*shape[1]*shape[2] elements of the
 * reported dtype), enqueued on the handle's stream and then synchronised.
 * Same arguments and errors as tnrsvd_get_factor; dst must not be NULL.
 */
tnrsvd_status tnrsvd_copy_factor(tnrsvd_t h, int b, int which, int core, void* dst);

/*
 * tnrsvd_get_omega / tnrsvd_set_omega -- read or replace Omega of MPO b in
 * FP64, as the concatenation omega_0 (J_0 values), ..., omega_{d'-2}, then
 * the J_{d'-1} x K matrix of the merged core in C order; *n (get) receives
 * the count, d' being the merged core count.  set_omega copies host_in
 * (that many doubles) to the device and synchronises the stream.
 */
tnrsvd_status tnrsvd_get_omega(tnrsvd_t h, int b, double* host_out, int64_t* n);
tnrsvd_status tnrsvd_set_omega(tnrsvd_t h, int b, const double* host_in);

/*
 * tnrsvd_get_ranks -- bond ranks of the current basis of MPO b: d'+1 values
 * r_0 = 1, ..., r_{d'} = K written to host_out (synchronises the stream).
 * *d_merged receives d'.
 */
tnrsvd_status tnrsvd_get_ranks(tnrsvd_t h, int b, int64_t* host_out, int* d_merged);

/*
 * Measurement aids.
 *
 * tnrsvd_profile -- enable (nonzero) or disable (0) per-launch timing: while
 * enabled, every kernel launch of the handle is bracketed by two HIP events
 * recorded on the handle's stream.  Enabling clears earlier records.
 * tnrsvd_profile_read -- synchronise the stream and return, for one kernel
 * kind, the summed event time (ms) and the launch count since enabling.
 * Kernel kinds: 0 contraction (Sec. 5.2 products), 1 right-to-left LQ sweep,
 * 2 left-to-right truncation/QR/SVD sweep, 3 U = Q W, 4 Omega load, 5 Y copy,
 * 6 sketched product truncation (opts.sketch_rank > 0).
 * tnrsvd_get_product_ranks -- product ranks P_0..P_d (P_d = K) of the last
 * product and the ranks rho_0..rho_d left by its right-to-left sweep (valid
 * after the sweep); synchronises the stream.  Either pointer may be NULL.
 */
tnrsvd_status tnrsvd_profile(tnrsvd_t h, int enable);
tnrsvd_status tnrsvd_profile_read(tnrsvd_t h, int kernel, double* total_ms, int64_t* launches);
tnrsvd_status tnrsvd_get_product_ranks(tnrsvd_t h, int b, int64_t* P_out, int64_t* rho_out);

/*
 * tnrsvd_sparse_to_mpo -- Algorithm 4.1 (Sec. 4.1): the MPO of a sparse
 * matrix A (M x N, M = prod rows[k], N = prod cols[k]) given by nnz entries
 * in COO form, with the mode sizes rows[0..d-1], cols[0..d-1] (HOST arrays)
 * and the little-endian index ordering of eq. (1): row i = i_1 + I_1 (i_2 +
 * I_2 (...)), so the first core carries the fastest index.  A is split into
 * I_1 x J_1 blocks; every block with a nonzero entry becomes one rank-1 term
 * (X, E^(2), ..., E^(d)), E^(k) being the unit matrix of the block's k-th
 * row and column digits, and the terms are added, so the MPO rank is the
 * number of nonzero blocks (the rank lemma of Sec. 4.2):
 *   core 0 (1, I_1, J_1, R):  [0, x, y, t] = X_t[x, y]
 *   core k (R, I_k, J_k, R):  [t, i_k(t), j_k(t), t] = 1   (0 < k < d-1)
 *   core d-1 (R, I_d, J_d, 1): [t, i_d(t), j_d(t), 0] = 1
 * (a single core, d = 1, is A itself).  Blocks t are numbered in increasing
 * order of (i / I_1) * (N / J_1) + (j / J_1).  Explicit zeros form no block;
 * duplicate entries add (atomically: their summation order is not fixed);
 * the zero matrix gives one all-zero rank-1 term (R = 1).
 * coo_row, coo_col (int64), coo_val (double): DEVICE arrays of nnz entries,
 *   in any order; each index must lie in [0, M) resp. [0, N).
 * Two calls.  With cores == NULL, *nblocks receives R.  With cores != NULL,
 *   *nblocks must hold that R on input, cores holds d DEVICE pointers to
 *   caller-allocated FP64 buffers of the shapes above in C order, which are
 *   overwritten in full; the count is recomputed and nothing is written if it
 *   differs from *nblocks.
 * stream: the hipStream_t to run on (NULL: the null stream); the call
 *   allocates and frees its own scratch and synchronises the stream.
 * Errors: E_INVALID (null array, *nblocks < 1 with cores); E_SHAPE (d < 1,
 * a mode size < 1, nnz outside [0, 2^31), dimensions or block positions
 * beyond 2^62, an index outside the matrix, a block count that differs
 * from *nblocks: no core written); E_DEVICE.
 */
tnrsvd_status tnrsvd_sparse_to_mpo(int d, const int64_t* rows, const int64_t* cols, int64_t nnz,
                                   const int64_t* coo_row, const int64_t* coo_col,
                                   const double* coo_val, int64_t* nblocks, double* const* cores,
                                   void* stream);

/*
 * tnrsvd_sparse_to_mpo_noalloc -- tnrsvd_sparse_to_mpo for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same two calls, arguments, results
 * and errors, on the same kernels, but the scratch (block bitmap or sort
 * keys, prefix sums, counters, the unit-entry table and the prefix-sum /
 * sort temporaries) lives in a file-scope device array of the library
 * (32 MiB, kNoAllocScratchBytes; each GPU the library runs on holds its own
 * copy until the process ends).  No hipMalloc, hipFree or allocating library
 * routine is called; the caller still passes inputs and cores.
 * Limits: inputs whose scratch exceeds 32 MiB (about 8.9e7 block positions on
 *   the bitmap path, 6e5 entries on the sort path) and d > 64 return E_SHAPE
 *   with the size needed.  Device ordinals 0..63.
 * Every call on one GPU shares that GPU's array and leaves its contents
 *   behind; the call clears what must start at zero.  Calls are serialised
 *   within a process (each ends with a stream synchronisation); calls that
 *   overlap on one GPU from elsewhere would race on the array.
 */
tnrsvd_status tnrsvd_sparse_to_mpo_noalloc(int d, const int64_t* rows, const int64_t* cols,
                                           int64_t nnz, const int64_t* coo_row,
                                           const int64_t* coo_col, const double* coo_val,
                                           int64_t* nblocks, double* const* cores, void* stream);

/*
 * tnrsvd_sparse_round -- the SVD-based rounding of Sec. 3 applied to the MPO
 * that Algorithm 4.1 (tnrsvd_sparse_to_mpo) builds from the same COO input,
 * computed without forming that MPO.  The rounding is the one the paper uses
 * on its converted matrices (Sec. 6.1): orthogonalise right to left, then
 * truncate left to right with singular-value tail delta = round_tol * |A|_F /
 * sqrt(d - 1) per bond (ranks capped at max_rank when max_rank > 0, and >= 1).
 * Result, in C order: core 0 (1, I_1, J_1, r_1), core k (r_k, I_k, J_k,
 * r_{k+1}), last core (r_{d-1}, I_d, J_d, 1); cores 0..d-2 are
 * left-orthonormal, with each left singular vector signed so that its entry
 * of largest magnitude (the first on ties) is positive, and the last core
 * carries the rest.  Since the selection cores orthogonalise exactly, only the
 * first core's truncated SVD is large (I_1 J_1 x R, R nonzero blocks): it runs
 * as a TSQR over all CUs; every later core is one small SVD.
 * Arguments as tnrsvd_sparse_to_mpo.  The zero matrix gives all-zero rank-1
 * cores; d = 1 gives the matrix itself.  Limits: at most 2^28 block
 * positions (I / I_1)(J / J_1), 16384 nonzero blocks, and I_1 J_1 < 2^31.
 * Rows of the first core without any nonzero entry add nothing to its R
 * factor and get zero rows in the result, so the TSQR runs over the others.
 * stream: hipStream_t (NULL: null stream); the call allocates its own
 * workspace, frees it, and synchronises the stream.
 * *out receives a handle owning the rounded cores (device memory) until
 * tnrsvd_rounded_destroy.  tnrsvd_rounded_ranks writes the d + 1 ranks
 * r_0 = 1, ..., r_d = 1 (HOST array).  tnrsvd_rounded_copy copies core k into
 * the DEVICE buffer dst (r_k I_k J_k r_{k+1} doubles) and synchronises.
 * Errors: E_INVALID (null argument, round_tol negative or not finite,
 * max_rank < 0, k out of range); E_SHAPE (as tnrsvd_sparse_to_mpo, or a
 * limit above exceeded); E_DEVICE.
 */
tnrsvd_status tnrsvd_sparse_round(int d, const int64_t* rows, const int64_t* cols, int64_t nnz,
                                  const int64_t* coo_row, const int64_t* coo_col,
                                  const double* coo_val, double round_tol, int max_rank,
                                  void* stream, tnrsvd_rounded_t* out);
/*
 * tnrsvd_round_mpo -- SVD-based rounding (Sec. 3) of any MPO a (device cores
 * (r, I, J, r'), FP64 or FP32; FP32 is widened, all arithmetic is FP64).
 * Core k is read as the (r_k) x (I_k J_k) x (r_{k+1}) core of an MPS (row
 * and column index grouped, the row index slower).  Right to left, the LQ
 * of each core k >= 2 (QR with diag(R) >= 0 of its transpose) leaves it with
 * orthonormal rows and L goes into the left neighbour; then
 * delta = round_tol |A|_F / sqrt(d - 1) and, left to right, the truncated SVD
 * of the carried factor times core k keeps the smallest rank whose
 * discarded singular values have squared sum <= delta^2 (capped at max_rank
 * when > 0); left vectors are sign-fixed (largest-magnitude entry positive)
 * and the last core carries the rest.  The result is left-orthonormal, and
 * the rounded matrix is within round_tol |A|_F of A in Frobenius norm.  The
 * zero matrix (|A|_F = 0) gives all-zero rank-1 cores; d = 1 gives the core.
 * a is read only; the call allocates its own workspace, frees it, and
 * synchronises `stream` (hipStream_t, NULL: null stream).  Limits: ranks up to
 * 4096, and r I J and I J r' below 2^31 for every core.
 * *out receives a handle owning the rounded cores, read with
 * tnrsvd_rounded_ranks / tnrsvd_rounded_copy, freed by tnrsvd_rounded_destroy.
 * Errors: E_INVALID (null argument, dtype, round_tol negative or not finite,
 * max_rank < 0); E_SHAPE (rank[0] or rank[d] not 1, a bad or too large
 * core); E_NOMEM; E_DEVICE.
 */
tnrsvd_status tnrsvd_round_mpo(const tnrsvd_mpo* a, double round_tol, int max_rank, void* stream,
                               tnrsvd_rounded_t* out);
/*
 * tnrsvd_complex_embed -- real form of a complex MPO (the paper allows real
 * or complex cores, Sec. 2; the embedding is a standard identity, not the
 * paper's).  a's cores are complex, stored as interleaved (re, im) pairs of
 * a->dtype (F64 or F32) in C order (R, I, J, R'); a->rank/rows/cols are
 * the complex MPO's.  Every bond entry z becomes the 2 x 2 block
 * phi(z) = [[Re z, -Im z], [Im z, Re z]] (phi(xy) = phi(x) phi(y)), bond index
 * (a, s) -> 2 a + s, so the inner ranks double; the first core's left
 * component becomes the most significant digit of its row mode (I_1 -> 2 I_1)
 * and the last core's right component that of its column mode (J_d -> 2 J_d).
 * The result B is a row and column permutation of [[Re A, -Im A], [Im A,
 * Re A]]: its singular values are A's, each twice, so TNrSVD of B with k' = 2k
 * and p' = 2p, every other value taken, solves A.  out[k]: caller-allocated
 * DEVICE buffers of the real core k, (2R or 1) x (2I or I) x (2J or J) x
 * (2R' or 1) elements of a->dtype.  Synchronises `stream`.
 * Errors: E_INVALID (null argument, dtype), E_SHAPE (ranks, shapes), E_DEVICE.
 */
tnrsvd_status tnrsvd_complex_embed(const tnrsvd_mpo* a, void* const* out, void* stream);
/*
 * tnrsvd_solve_complex -- top-k singular values of a complex MPO in one call
 * (cores allowed complex in Sec. 2; the embedding is not the paper's): the
 * real form of tnrsvd_complex_embed, in device buffers this call allocates
 * and frees, solved by tnrsvd_run with k' = 2 opts->k and p' = 2 opts->p
 * (each value of A appears twice in the real form), every other value
 * returned.  a: as for tnrsvd_complex_embed; opts: the complex problem's
 * options (k, p of A; q, seed, precision, tolerance, rank cap, stream,
 * orientation and sketch rank as for tnrsvd_create, applied to the real
 * form); sigma: HOST array of opts->k doubles, descending.  Synchronises the
 * stream.  Errors: those of tnrsvd_complex_embed, tnrsvd_create (with k' and
 * p') and tnrsvd_run; E_INVALID (null argument, opts->k < 1, opts->p < 0).
 */
tnrsvd_status tnrsvd_solve_complex(const tnrsvd_mpo* a, const tnrsvd_opts* opts, double* sigma);
/*
 * tnrsvd_mpo_add -- the MPO of the sum of two matrices given as MPOs with the
 * same row and column modes (Sec. 3: ranks add).  a and b: device cores
 * (r, I, J, r') of the same dtype (F64 or F32), rank[0] = rank[d] = 1.  The
 * sum C has ranks 1, ra_1 + rb_1, ..., ra_{d-1} + rb_{d-1}, 1: its first core
 * is [A_1 B_1] along the right rank leg, its last core [A_d; B_d] along the
 * left one, and every inner core is block diagonal, diag(A_k, B_k), with
 * zeros elsewhere; for d = 1 the single core is A_1 + B_1.  Entries are
 * copied exactly (d = 1: one correctly rounded addition).  The ranks are not
 * reduced: tnrsvd_round_mpo rounds the sum.  out[k]: caller-allocated DEVICE
 * buffer of core k of C, ((k = 0) ? 1 : ra_k + rb_k) x I_k x J_k x
 * ((k = d-1) ? 1 : ra_{k+1} + rb_{k+1}) elements in C order; a and b are
 * read only.  Synchronises `stream` (hipStream_t, NULL: null stream).
 * Errors: E_INVALID (null argument, dtype), E_SHAPE (d or modes differ, end
 * ranks not 1, a rank below 1, a core of C with 2^40 entries or more or a
 * rank above 2^20), E_DEVICE.
 */
tnrsvd_status tnrsvd_mpo_add(const tnrsvd_mpo* a, const tnrsvd_mpo* b, void* const* out,
                             void* stream);
tnrsvd_status tnrsvd_rounded_ranks(tnrsvd_rounded_t r, int64_t* ranks);
tnrsvd_status tnrsvd_rounded_copy(tnrsvd_rounded_t r, int k, double* dst);
tnrsvd_status tnrsvd_rounded_destroy(tnrsvd_rounded_t r);

/* tnrsvd_destroy -- free every device buffer of the handle (NULL is a no-op). */
tnrsvd_status tnrsvd_destroy(tnrsvd_t h);

/* Message of the last failing call on this thread ("" if none). */
const char* tnrsvd_last_error(void);

/* Library version string. */
const char* tnrsvd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TNRSVD_H */
