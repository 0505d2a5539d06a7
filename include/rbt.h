/*
 * rbt.h - C ABI of the MI355X (gfx950) generalized random butterfly
 * transform (RBT) solver.
 *
 * Method: Lindquist, Luszczek, Dongarra, "Generalizing Random Butterfly
 * Transforms to Arbitrary Matrix Sizes" (ACM TOMS; arXiv 2312.09376).
 * A x = b is rewritten as (U^T A V)(V^-1 x) = U^T b (Sec. 1, Eq. 1); the
 * transformed matrix is factored by Gaussian elimination with no pivoting
 * (GENP), the two triangular systems are solved and x = V x~ is recovered.
 * U and V are depth-d generalized (semi-Parker) RBTs (Sec. 3, Eq. 2-4)
 * truncated to any n.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major. Element (i, j) of A is A[i + j * lda].
 *   - Sizes and leading dimensions are int64_t; a leading dimension must be
 *     >= max(1, rows).
 *   - Pointers named d* or documented as "device" point to device memory
 *     (hipMalloc'd or torch CUDA/HIP tensors); the caller owns all memory.
 *     The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Device
 *     work is enqueued asynchronously on it; the entry point returns after
 *     enqueueing unless documented otherwise.
 *   - Return value: 0 on success; -i if argument i (1-based) is invalid (the
 *     check is synchronous and nothing is enqueued); RBT_ERR_HIP if a HIP
 *     runtime call failed; RBT_ERR_WORKSPACE if the workspace is too small;
 *     RBT_ERR_UNSUPPORTED for a configuration the library does not implement.
 *   - Packed coefficients: U and V are n x depth FP64 arrays (ld = n) whose
 *     column k is the diagonal of R_{k+1} (Sec. 3, packed storage of Alg. 1).
 *     Layer 1 is the single full-size butterfly of Eq. 3.
 *   - Butterfly structure: non-tiled reference size m = 2^d ceil(n/2^d)
 *     (Sec. 3, after Alg. 1) and global half-sizes h_l = m / 2^l in layer l.
 *     In layer l, index i pairs with i + h_l (top half) or i - h_l (bottom
 *     half) when that index is < n; otherwise it is unpaired and only scaled
 *     (Eq. 2: factor 1, not 1/sqrt 2).
 *   - Coefficients are exp(r/20), r uniform on [-1, 1) (Sec. 6 setup), drawn
 *     from a counter-based SplitMix64 stream (Steele, Lea, Flood 2014):
 *     draw(seed, c) = SplitMix64 output number c from state `seed`,
 *     c = 128 i + 64 side + (layer - 1), side 0 = U, 1 = V;
 *     r = 2 (draw >> 11) 2^-53 - 1.
 */
#ifndef RBT_H
#define RBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBT_ERR_HIP (-100)
#define RBT_ERR_WORKSPACE (-101)
#define RBT_ERR_UNSUPPORTED (-102)
/* A persistent triangular sweep waited longer than its bound for a block
 * that another workgroup had to publish (device oversubscribed or starved).
 * The blocks solved after the expired wait are NaN, never silently wrong
 * finite values; entry points that synchronize return this code, the others
 * leave the NaN in their output. */
#define RBT_ERR_SYNC (-103)

/* Largest supported depth. */
#define RBT_MAX_DEPTH 16

/* Precision of the factorization. */
#define RBT_FP64 0
#define RBT_FP32 1
#define RBT_BF16 2

/* Direction of a one-sided butterfly application. */
#define RBT_OP_T 0 /* B <- C^T B : forward side (b~ = U^T b, Eq. 1) */
#define RBT_OP_N 1 /* B <- C B   : undo side (x = V x~, Eq. 1)       */

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int rbt_version(void);

/* Host only. Butterfly structure, for inspection and tests.
 * partner: host array of n * depth int64; on return partner[(l-1) * n + i]
 * is the index paired with i in layer l, or -1 if i is unpaired there
 * (Sec. 3, Eq. 2-4, Alg. 1 loop nest). n >= 0, 0 <= depth <= RBT_MAX_DEPTH. */
int rbt_structure(int64_t n, int depth, int64_t *partner);

/* Host only. Reference size m = 2^d g ceil(n / (2^d g)) of the butterfly
 * structure for the granule g >= 1 (Sec. 3, text after Alg. 1): g = 1 is the
 * non-tiled size, g = n_b aligns every butterfly to n_b x n_b tiles, and
 * g = rbt_comm_free_granule(n_b, p, q) is the size of Eq. 8 (Sec. 6.4).
 * -1 for invalid arguments. */
int64_t rbt_reference_size(int64_t n, int depth, int64_t granule);

/* Host only. Granule of the communication-free size of Eq. 8 (Sec. 6.4):
 * lcm(p, q) * nb for a p x q process grid of nb x nb tiles. With it every
 * pair of every layer lies on one process row (U side) and one process
 * column (V side) of a 2-D block-cyclic distribution. -1 for invalid
 * arguments. */
int64_t rbt_comm_free_granule(int64_t nb, int64_t p, int64_t q);

/* Host only. rbt_structure for the reference size of granule `granule`
 * (argument 3; partner is argument 4). The device entry points use the
 * granule set with rbt_set_option(RBT_OPT_GRANULE, g) (default 1). */
int rbt_structure_ex(int64_t n, int depth, int64_t granule, int64_t *partner);

/* Host only. Packed coefficients U, V (host arrays of n * depth doubles each,
 * column-major, ld = n) for (n, depth, seed), per the generator above.
 * Index i's coefficient in layer l depends only on (seed, side, l, i). */
int rbt_generate(int64_t n, int depth, uint64_t seed, double *U, double *V);

/* Host only. Packed coefficients of the rotation butterflies (Sec. 3: the
 * block-rotation form [[C, 0, S], [0, I, 0], [S, 0, -C]], C^2 + S^2 = I, a
 * rotation by 0 degrees on the truncated part, R_l = I) for the structure
 * of (n, depth, granule): for a pair (a, b) of layer l (a in the top half)
 * U[(l-1) n + a] = cos(theta), U[(l-1) n + b] = sin(theta), and 1 for an
 * unpaired index; theta = 2 pi u with u the uniform of the coefficient
 * counter at the top index (side 0 for U, 1 for V). */
int rbt_generate_rotations(int64_t n, int depth, uint64_t seed, int64_t granule, double *U,
                           double *V);

/* Device. Same coefficients written to device arrays dU, dV (n * depth
 * doubles each); exp is the device library's, within 2 ulp of the host's.
 * With RBT_OPT_BUTTERFLY = 1 the rotation coefficients (cos and sin from
 * the device library) of the current granule. */
int rbt_generate_device(int64_t n, int depth, uint64_t seed, double *dU, double *dV,
                        void *stream);

/* Device. Two-sided transform Out = U^T A V (Eq. 1), all depth layers in
 * one pass over HBM for depth <= 3 (the single-pass fusion suggested at the
 * end of Sec. 3), ceil(depth / 3) passes otherwise.
 * A: n x n FP64 (lda); Out: n x n (ldo) of type out_prec (RBT_FP64 or
 * RBT_FP32). Out may equal A (in place) only when out_prec == RBT_FP64 and
 * ldo == lda. dU, dV: packed device coefficients. */
int rbt_transform2(int64_t n, const double *A, int64_t lda, void *Out, int64_t ldo, int out_prec,
                   const double *dU, const double *dV, int depth, void *stream);

/* Device. One-sided transform of an n x nrhs FP64 block B (ldb), in place:
 * op = RBT_OP_T: B <- C^T B (layers d..1: mix, then scale);
 * op = RBT_OP_N: B <- C B   (layers 1..d: scale, then mix).
 * dC: packed device coefficients (U or V). */
int rbt_transform_vec(int64_t n, int64_t nrhs, double *B, int64_t ldb, const double *dC, int depth,
                      int op, void *stream);

/* Workspace (bytes) needed by rbt_getrs / rbt_solve_ex / rbt_solve_refine /
 * rbt_backward_error (precision RBT_FP64) or rbt_solve_mixed (RBT_FP32,
 * RBT_BF16) for these sizes (0 for invalid arguments). */
size_t rbt_workspace_size(int64_t n, int64_t nrhs, int depth, int precision);

/* Device. GENP of the n x n FP64 matrix A (lda) in place: unit-lower L
 * strictly below the diagonal, U on and above (Sec. 1, step 2; no pivoting,
 * no perturbation). Blocked right-looking with 128 x 128 diagonal blocks.
 * info_dev (device int32, nullable) receives 0 or k > 0 when U(k,k) is
 * exactly zero (1-based, first such k); the elimination goes on with IEEE
 * Inf/NaN. */
int rbt_genp(int64_t n, double *A, int64_t lda, int32_t *info_dev, void *stream);

/* Device. Solve with the factors of rbt_genp: trans = 0: B <- (L U)^-1 B;
 * trans = 1: B <- (L U)^-T B. B: n x nrhs FP64 (ldb), in place.
 * work: device scratch of rbt_workspace_size(n, nrhs, 0, RBT_FP64) bytes
 * (for nrhs <= 16 it receives the inverses of the 128 x 128 diagonal blocks,
 * which the solve applies with one step of refinement per block). */
int rbt_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu, double *B, int64_t ldb,
              int trans, void *work, size_t work_bytes, void *stream);

/* Device. The whole method (Eq. 1): A (n x n, lda) is overwritten by the
 * L\U factors of A~ = U^T A V, B (n x nrhs, ldb) by X = A^-1 B. Coefficients
 * are generated on the device from (depth, seed). info_dev: as rbt_genp.
 * work: >= rbt_workspace_size(n, nrhs, depth, RBT_FP64) bytes; on return
 * it holds U, V and the factor data needed by rbt_solve_backward. */
int rbt_solve_ex(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb, int depth,
                 uint64_t seed, int32_t *info_dev, void *work, size_t work_bytes, void *stream);

/* Device. rbt_solve_ex for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument, and no allocation or allocating library call. The
 * workspace is a library-owned device array of RBT_NOALLOC_SCRATCH_MB MiB on
 * each GPU the library runs on (held until the process ends; its address is
 * looked up once per device on the first call there). Sizes whose workspace
 * rbt_workspace_size(n, nrhs, depth, RBT_FP64) exceeds it return
 * RBT_ERR_WORKSPACE (n <= 28000 or so with one right-hand side, about
 * 9000 with sixteen). Every
 * call on one GPU uses the same array: calls that overlap on one GPU (other
 * streams, other threads) race; the array keeps the last call's contents and
 * the solve writes every part it reads. Arguments and results as
 * rbt_solve_ex (work and work_bytes omitted). */
#define RBT_NOALLOC_SCRATCH_MB 96
int rbt_solve_ex_noalloc(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                         int depth, uint64_t seed, int32_t *info_dev, void *stream);

/* Device. As rbt_solve_ex, but the library allocates its workspace with
 * hipMallocAsync/hipFreeAsync on `stream`. */
int rbt_solve(int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb, int depth,
              uint64_t seed, void *stream);

/* Device. The method with stationary iterative refinement in FP64
 * (Sec. 5): A (n x n, lda) is read only and kept for the residuals; LU
 * (n x n, ldlu) receives the factors of A~; X (n x nrhs, ldx) receives the
 * solution of A X = B (B: n x nrhs, ldb, read only). Refinement steps
 * X += V (LU)^-1 U^T (B - A X) run until the backward error of Eq. 7
 * (infinity norms, maximum over columns) is <= tol or max_iter steps are
 * done. iters_dev (device int32) and berr_dev (device double) receive the
 * step count and the final backward error (both nullable). This entry point
 * synchronizes `stream` once per refinement step to test convergence,
 * unless RBT_OPT_CAPTURABLE is set (then it never synchronizes). */
int rbt_solve_refine(int64_t n, int64_t nrhs, const double *A, int64_t lda, double *LU,
                     int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx, int depth,
                     uint64_t seed, double tol, int max_iter, int32_t *iters_dev, double *berr_dev,
                     int32_t *info_dev, void *work, size_t work_bytes, void *stream);

/* Refinement schemes of rbt_solve_mixed. */
#define RBT_IR_CLASSIC 0 /* X += V (LU)^-1 U^T (B - A X)                         */
#define RBT_IR_GMRES 1   /* correction by GMRES on A, preconditioned by V (LU)^-1 U^T */

/* Device. Mixed-precision form of rbt_solve_refine (the refinement of Sec. 5
 * with a factorization in lower precision, the mixed-precision refinement
 * the paper points to in its discussion of accuracy): A (n x n FP64, lda) is
 * read only and kept for the residuals; A~ = U^T A V is formed from it in
 * FP64 arithmetic and stored in FP32 into LU (n x n FP32, ldlu), which is
 * then eliminated without pivoting in place:
 *   prec = RBT_FP32: FP32 storage, FP32 matrix-core updates;
 *   prec = RBT_BF16: FP32 storage, updates with operands rounded to BF16
 *                    (nearest even) and FP32 accumulation.
 * The whole elimination is FP32 arithmetic (diagonal blocks and panel
 * solves too). With classical refinement, so are the two triangular solves
 * with the FP32 factors inside each correction (the transformed residual is
 * rounded to FP32, the result widened); GMRES-IR applies its preconditioner
 * V (LU)^-1 U^T in FP64 arithmetic on the FP32 factors, the working
 * precision in which that method defines the preconditioned products.
 * RBT_OPT_MIXED_FP64_INNER selects FP64 arithmetic for all of those inner
 * steps. Refinement is in FP64 with the original A:
 *   solver = RBT_IR_CLASSIC: X += V (LU)^-1 U^T (B - A X);
 *   solver = RBT_IR_GMRES:   the correction solves A D = B - A X by restarted
 *                            GMRES in FP64, preconditioned on the left by
 *                            V (LU)^-1 U^T.
 * Stops when the Eq. 7 backward error is <= tol or after max_iter
 * corrections (GMRES: iterations of the Krylov method). iters_dev, berr_dev,
 * info_dev: as rbt_solve_refine. depth <= RBT_MAX_DEPTH; beyond depth 3 the
 * FP32 A~ is rounded to FP32 after every pass of three layers.
 * work: >= rbt_workspace_size(n, nrhs, depth, prec) bytes. Synchronizes
 * `stream` once per refinement step. */
int rbt_solve_mixed(int64_t n, int64_t nrhs, const double *A, int64_t lda, float *LU,
                    int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx, int depth,
                    uint64_t seed, int prec, int solver, double tol, int max_iter,
                    int32_t *iters_dev, double *berr_dev, int32_t *info_dev, void *work,
                    size_t work_bytes, void *stream);

/* Device. rbt_solve_mixed with a fallback to FP64 factors: try the
 * low-precision factors first and, only if their refinement cannot reach
 * tol, factor A~ again in FP64 and refine with those. Sec. 5 pairs the
 * fast unpivoted solve with a check of its result and re-solves with a more
 * robust solver only when refinement fails; here the more robust solve is
 * the same method in FP64 (same butterflies, FP64 GENP, classical FP64
 * refinement): this library has no pivoted factorization.
 *
 * The low-precision phase is rbt_solve_mixed with max_iter as its budget,
 * except that it also stops early when tol is out of reach: a non-finite
 * backward error; classical: a correction that does not halve the backward
 * error; GMRES: from the 8th iteration of a cycle on, when the residual
 * estimate, extrapolated at the geometric rate of its last 4 iterations
 * over the remaining budget, leaves the backward error > 1e3 * tol. The
 * fallback then runs when the final
 * backward error is not <= tol (NaN included), with at most max_iter64
 * classical corrections, which stop early in the same way. If those cannot
 * reach tol either (the transform itself fails on this matrix, as for the
 * `orthog` matrix of Sec. 6.3), A is re-solved with partial pivoting
 * (rbt_gepp) into LU64 and refined with those factors (max_iter64
 * corrections): the more robust solver Sec. 5 names.
 *
 * LU64: n x n FP64 (ldlu64 >= max(1, n)), caller-owned, written only by a
 * fallback (then it holds the FP64 factors of A~). Other arguments as in
 * rbt_solve_mixed; work: rbt_workspace_size(n, nrhs, depth, prec) bytes.
 * iters_dev: device int32[2] = {low-precision iterations, FP64
 * corrections}; info_dev: device int32[2] = {info of the low-precision
 * elimination, info of the FP64 one (0 without fallback)}; path_dev: device
 * int32, 0 = low-precision factors reached tol, 1 = FP64 RBT fallback,
 * 2 = partial-pivoting re-solve (info_dev[1] then holds its zero-pivot
 * column, iters_dev[1] its corrections);
 * berr_dev: final Eq. 7 backward error. All four nullable. Synchronizes
 * `stream` as rbt_solve_mixed does, and once more before returning.
 * Errors: -i for argument i; RBT_ERR_WORKSPACE; RBT_ERR_HIP. */
int rbt_solve_mixed_guarded(int64_t n, int64_t nrhs, const double *A, int64_t lda, float *LU,
                            int64_t ldlu, double *LU64, int64_t ldlu64, const double *B,
                            int64_t ldb, double *X, int64_t ldx, int depth, uint64_t seed,
                            int prec, int solver, double tol, int max_iter, int max_iter64,
                            int32_t *iters_dev, double *berr_dev, int32_t *info_dev,
                            int32_t *path_dev, void *work, size_t work_bytes, void *stream);

/* Device. Elimination with partial pivoting (GEPP) of the n x n FP64 matrix
 * A (lda) in place: P A = L U, unit-lower L strictly below the diagonal, U
 * on and above; ipiv_dev (device int64[n]) receives the 1-based row
 * interchanges in order (LAPACK getrf's convention); info_dev (device int32,
 * nullable): 0, or the first column k (1-based) whose pivot candidates were
 * all exactly zero (left unswapped; the elimination goes on with IEEE
 * Inf/NaN). This is the robust solver that the fallback of Sec. 5 re-solves
 * with. work: >= rbt_workspace_size(n, 0, 0, RBT_FP64) bytes. */
int rbt_gepp(int64_t n, double *A, int64_t lda, int64_t *ipiv_dev, int32_t *info_dev, void *work,
             size_t work_bytes, void *stream);

/* Device. B <- A^-1 B (n x nrhs FP64, ldb, in place) with the factors and
 * interchanges of rbt_gepp. work: >= rbt_workspace_size(n, nrhs, 0,
 * RBT_FP64) bytes. */
int rbt_gepp_solve(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu,
                   const int64_t *ipiv_dev, double *B, int64_t ldb, void *work, size_t work_bytes,
                   void *stream);

/* Device. The FP64 method with its Sec. 5 fallback: rbt_solve_refine, whose
 * refinement stops early when tol is out of reach (a non-finite backward
 * error, or a correction that does not halve it), and, if the backward error
 * is then not <= tol, a re-solve of A with partial pivoting (rbt_gepp) into
 * LU with max_iter classical FP64 corrections. Arguments as rbt_solve_refine;
 * iters_dev: device int32[2] = {RBT corrections, pivoted corrections};
 * info_dev: device int32[2] = {first zero pivot of GENP on A~, first zero
 * pivot column of GEPP}; path_dev: device int32, 0 = the RBT solve reached
 * tol, 2 = the pivoted re-solve ran. All four nullable. work: >=
 * rbt_workspace_size(n, nrhs, depth, RBT_FP64) bytes. Synchronizes `stream`
 * once per refinement step and before returning. */
int rbt_solve_guarded(int64_t n, int64_t nrhs, const double *A, int64_t lda, double *LU,
                      int64_t ldlu, const double *B, int64_t ldb, double *X, int64_t ldx,
                      int depth, uint64_t seed, double tol, int max_iter, int32_t *iters_dev,
                      double *berr_dev, int32_t *info_dev, int32_t *path_dev, void *work,
                      size_t work_bytes, void *stream);

/* Batched solves: many independent systems A_s X_s = B_s of different
 * orders (the method of Eq. 1 per system, with mixed precision as in
 * rbt_solve_mixed: FP32 elimination of A~_s, or BF16 trailing-update
 * operands, and classical FP64 refinement with the original A_s), all in ONE
 * persistent launch: each workgroup takes systems from a queue, largest
 * first, and runs every step of the method on each. A system whose
 * low-precision refinement does not reach tol is factored again with FP64
 * storage and arithmetic (same coefficients) and refined again.
 *
 * Host. Workspace bytes for a batch of `batch` systems with orders n[s] and
 * right-hand-side counts nrhs[s] (host arrays; 0 <= nrhs[s] <= 16), depth
 * <= RBT_MAX_DEPTH, prec RBT_FP32 or RBT_BF16; 0 for invalid arguments. About
 * 12 n^2 + 8 (2 n d + 64^2 ceil(n/64) + n nrhs) bytes per system (FP32
 * factors, FP64 factors of the fallback, coefficients, inverse blocks,
 * residual). */
size_t rbt_batched_workspace_size(int64_t batch, const int64_t *n, const int64_t *nrhs, int depth,
                                  int prec);

/* Host. Write the plan (header and queue of systems, largest first) for
 * these sizes into the device workspace `work` (>= rbt_batched_workspace_size
 * bytes); synchronizes `stream`. Call once per set of sizes; the plan stays
 * valid for any number of rbt_solve_batched calls with the same batch,
 * depth and prec. nrhs[s] > 16: RBT_ERR_UNSUPPORTED. Each system's
 * transforms run in passes of at most three layers. */
int rbt_batched_plan(int64_t batch, const int64_t *n, const int64_t *nrhs, int depth, int prec,
                     void *work, size_t work_bytes, void *stream);

/* Device. Solve the planned batch. A, lda, B, ldb, X, ldx: device arrays of
 * `batch` entries (pointers to column-major FP64 matrices in device memory
 * and their leading dimensions): A[s] n x n (read only, kept for the
 * residuals), B[s] n x nrhs (read only), X[s] n x nrhs (output). System s
 * draws its coefficients from seed_s = SplitMix64 output number s of `seed`
 * (the draw of the header's conventions, per system). Refinement stops per
 * system at the Eq. 7 backward error <= tol or after max_iter corrections;
 * tol < 0 means |tol| n_s 2^-52 for system s of order n_s (NaN: -11).
 * A system also stops when two corrections in a row fail to reduce its best
 * backward error by 10 % (stagnation), or when the error is NaN; its
 * berr_dev entry then stays above tol.
 * iters_dev, berr_dev, info_dev, path_dev: device arrays of `batch`
 * entries (nullable) for the correction count (both passes), the final
 * backward error, the first zero pivot (as rbt_genp) of the last pass, and
 * the pass that produced X (0: low precision, 1: FP64 fallback). Systems with
 * n = 0 or nrhs = 0 have nothing to solve and are not factored: iters 0,
 * berr 0, info 0, path 0. Enqueues a reset kernel and
 * the persistent kernel on `stream`, allocates nothing and synchronizes
 * nothing, so it can be captured in a HIP graph. A plan that does not match
 * (batch, depth, prec) or a workspace smaller than the plan's solves no
 * system and marks every one: info -1, berr NaN, path -1 (X untouched).
 * Concurrent calls with the same workspace race. */
int rbt_solve_batched(int64_t batch, const double *const *A, const int64_t *lda,
                      const double *const *B, const int64_t *ldb, double *const *X,
                      const int64_t *ldx, int depth, uint64_t seed, int prec, double tol,
                      int max_iter, int32_t *iters_dev, double *berr_dev, int32_t *info_dev,
                      int32_t *path_dev, void *work, size_t work_bytes, void *stream);

/* Device. Backward error of Eq. 7 for n x nrhs X against A (n x n) and B:
 * max over columns of ||B - A X||_inf / (||A||_inf ||X||_inf + ||B||_inf),
 * written to berr_dev (device double). work: >= rbt_workspace_size(n, nrhs,
 * 0, RBT_FP64) bytes. */
int rbt_backward_error(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *X,
                       int64_t ldx, const double *B, int64_t ldb, double *berr_dev, void *work,
                       size_t work_bytes, void *stream);

/* Device. Adjoint of X = A^-1 B for a loss with dL/dX = G (all FP64,
 * column-major): dB = Lambda = A^-T G and dA = -Lambda X^T. With
 * A = U^-T A~ V^-1 (Eq. 1), A^-T = U A~^-T V^T, so Lambda is formed through
 * the same butterflies and the saved factors of A~: G^ = V^T G, solve
 * U_f^T Z = G^ then L^T W = Z, Lambda = U W.
 * LU: the L\U factors of A~ left by rbt_solve_ex (or the LU output of
 * rbt_solve_refine) for the same (depth, seed); X: the forward solution
 * (only read when dA != NULL); G: n x nrhs; dB: n x nrhs output (may not
 * alias G); dA: n x n output, nullable (skipped). work: >=
 * rbt_workspace_size(n, nrhs, depth, RBT_FP64) bytes. */
int rbt_solve_backward(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu, const double *X,
                       int64_t ldx, const double *G, int64_t ldg, double *dA, int64_t ldda,
                       double *dB, int64_t lddb, int depth, uint64_t seed, void *work,
                       size_t work_bytes, void *stream);

/* Device. Adjoint of the mixed-precision solve (rbt_solve_mixed): LU = the
 * FP32 L\U factors of A~ left by rbt_solve_mixed for the same (depth,
 * seed); A = the original FP64 matrix (n x n, lda), used to refine
 * Lambda = A^-T G in FP64: Lambda_0 = U (LU)^-T V^T G with the FP32 factors
 * (FP32 triangular solves, or FP64 ones with RBT_OPT_MIXED_FP64_INNER), then
 * Lambda += U (LU)^-T V^T (G - A^T
 * Lambda) until the Eq. 7 backward error of A^T Lambda = G (with
 * ||A^T||_inf = ||A||_1) is <= tol or max_iter corrections are done.
 * dB = Lambda, dA = -Lambda X^T (nullable: skipped). iters_dev, berr_dev:
 * as rbt_solve_refine. work: >= rbt_workspace_size(n, nrhs, depth,
 * RBT_FP32) bytes. Synchronizes `stream` once per correction. */
int rbt_solve_backward_mixed(int64_t n, int64_t nrhs, const float *LU, int64_t ldlu,
                             const double *A, int64_t lda, const double *X, int64_t ldx,
                             const double *G, int64_t ldg, double *dA, int64_t ldda, double *dB,
                             int64_t lddb, int depth, uint64_t seed, double tol, int max_iter,
                             int32_t *iters_dev, double *berr_dev, void *work, size_t work_bytes,
                             void *stream);

/* Tuning options (process-wide; not thread safe).
 * RBT_OPT_OUTER_NB: width of the panels of the elimination whose trailing
 *   update is a single GEMM (multiple of 128, 128..2048; default 2048). The
 *   first panel also takes the n mod 128 columns that do not fill a 128-wide
 *   diagonal block (except with BF16 updates), so that every trailing update
 *   covers whole 128-blocks. Changes only the order of the roundings, not
 *   the method. */
#define RBT_OPT_OUTER_NB 1
/* RBT_OPT_BATCH_TILE_COLS2_MIN_N: rbt_solve_batched, systems with
 *   n >= value take two 64-column tiles per round of the low-precision
 *   trailing update (fewer barriers and restagings of the row tile, more
 *   registers), smaller systems one (>= 0; default INT64_MAX: one for all).
 * RBT_OPT_BATCH_TILE_COLS: the same choice for every system (1: value
 *   INT64_MAX above, 2: value 0); reads 1 or 2, or 0 for a split by n.
 * RBT_OPT_BATCH_WGS_PER_CU: rbt_solve_batched, persistent workgroups per
 *   compute unit (1 or 2; default 2).
 * All change the schedule only: every system's arithmetic is the same. The
 * package's autotuner times the candidates (size thresholds at the bounds
 * of its n-buckets, workgroups per compute unit) on the device and keeps a
 * table per precision, which its binding applies before each launch; a
 * launch uses the values current when it is enqueued (or captured). */
#define RBT_OPT_BATCH_TILE_COLS 2
#define RBT_OPT_BATCH_WGS_PER_CU 3
#define RBT_OPT_BATCH_TILE_COLS2_MIN_N 12
/* RBT_OPT_LOOKAHEAD: elimination (rbt_genp and every solve that factors).
 *   1: while the next panel is factored on the caller's stream, the block
 *   row and trailing update of the remaining columns run on a second stream
 *   of the library (one per device, default priority, created on first
 *   use, ordered by HIP events; the caller's stream waits for it before the
 *   entry point returns). 0 (default): one stream. The factors are
 *   bit-identical either way. On MI355X the overlap gains little: the
 *   trailing GEMM's workgroups hold every CU's registers, so the panel
 *   kernels wait for its tiles to drain. */
#define RBT_OPT_LOOKAHEAD 4
/* RBT_OPT_BF16_STAGED: BF16 elimination (prec RBT_BF16), 1 (default): the
 *   trailing update rounds L21 and U12 to BF16 once into the workspace's
 *   staging area and runs the large-tile BF16 GEMM; 0: operands rounded
 *   tile by tile. Identical results. The staging area is part of
 *   rbt_workspace_size(..., RBT_BF16) at the panel width current when it is
 *   called; a smaller workspace (e.g. sized for RBT_FP32) or a wider panel
 *   selects the tile-by-tile path. */
#define RBT_OPT_BF16_STAGED 5
/* RBT_OPT_SWEEP_SPIN_LIMIT: sleeps (s_sleep 1, about 30 ns each) that a
 *   wait of a persistent triangular sweep may take before it expires
 *   (default 2^20). A negative value makes every wait expire at once: a
 *   host-side way to exercise the RBT_ERR_SYNC path in tests (every kernel
 *   still exits normally). */
#define RBT_OPT_SWEEP_SPIN_LIMIT 6
/* RBT_OPT_MIXED_FP64_INNER: low-precision elimination and solves
 *   (rbt_solve_mixed, rbt_solve_mixed_guarded, rbt_solve_backward_mixed).
 *   0 (default): the whole elimination of A~ is FP32 arithmetic (diagonal
 *   blocks, panel solves, FP32 or BF16-operand matrix-core updates with FP32
 *   accumulation) and so are the triangular solves of classical refinement
 *   with the FP32 factors (right-hand side rounded to FP32, result widened);
 *   FP64 is used only for the residual, the butterflies of the residual and
 *   correction, and the accumulation of x (and for GMRES-IR's
 *   preconditioner, which that method applies in the working precision).
 *   1: the diagonal blocks, panel solves and triangular solves run in FP64
 *   arithmetic on the FP32 factors (rounded to FP32 on store), a more
 *   accurate variant that is not FP32 elimination. */
#define RBT_OPT_MIXED_FP64_INNER 7
/* RBT_OPT_GRANULE: reference-size granule g of the butterfly structure used
 *   by every device entry point (transforms, solves, mixed, batched,
 *   adjoint): m = 2^d g ceil(n / (2^d g)). 1 (default): the non-tiled size;
 *   a tile size, or rbt_comm_free_granule(nb, p, q) for Eq. 8. Changes the
 *   transform (a different depth-d RBT), so factors and solutions saved
 *   under one granule must be used under the same granule. 1 .. 2^30. */
#define RBT_OPT_GRANULE 8
/* RBT_OPT_BUTTERFLY: kind of butterflies of every device entry point
 *   (coefficient draw, transforms, solves, mixed, batched, adjoint):
 *   0 (default): random diagonals R_l with the butterflies of Eq. 2 (Eq. 3);
 *   1: rotation butterflies (the block-rotation form of Sec. 3, R_l = I,
 *   orthogonal), coefficients as rbt_generate_rotations with the current
 *   granule. rbt_generate_device draws the coefficients of the current kind. */
#define RBT_OPT_BUTTERFLY 9
/* RBT_OPT_SIDES: 2 (default): A~ = U^T A V; 1: the one-sided RBT of Sec. 7,
 *   A~ = U^T A (columns untouched, x = x~; V is neither applied nor needed
 *   by the transforms, though the coefficient arrays keep their size). */
#define RBT_OPT_SIDES 10
/* RBT_OPT_CAPTURABLE: refinement of rbt_solve_refine and of rbt_solve_mixed
 *   with RBT_IR_CLASSIC (the stationary refinement of Sec. 5).
 *   0 (default): the host tests the Eq. 7 error after every step (one
 *   stream synchronization per step) and stops launching.
 *   1: no host test, synchronization or host-device copy in the call, so
 *   the call can be captured in a HIP graph: all max_iter steps are
 *   enqueued, and the kernels of a step return at once when a device word,
 *   set by the step's convergence test, says the error has reached tol.
 *   Same residuals, corrections, step count and final error as with 0;
 *   iters_dev is written on the device. Requires nrhs <= 16 (else
 *   RBT_ERR_UNSUPPORTED; also for RBT_IR_GMRES, whose small least-squares
 *   problems are solved on the host). An expired sweep wait is not reported
 *   as RBT_ERR_SYNC in this mode: the poisoned solution gives a NaN
 *   backward error. */
#define RBT_OPT_CAPTURABLE 11
/* RBT_OPT_PANEL_SPLIT: order of the work inside a panel of the elimination
 *   (every entry point that factors). 0: one 128-wide diagonal
 *   block after another, each followed by a depth-128 update of the panel's
 *   remaining columns and block rows. 1: recursive halves: the left half of
 *   the panel (whole 128-blocks) is factored first, then one update of
 *   depth = its width, then the right half, recursively down to 128. Every
 *   element receives the same updates, grouped into fewer, deeper products
 *   (a different order of the roundings, not a different method); the
 *   lookahead's block-row solves follow the same order, so the factors stay
 *   identical with and without lookahead. 2 (default): order 1 for panels
 *   with at least 8192 rows from their first row down, order 0 for the
 *   others (whose deeper updates have too few tiles to gain). */
#define RBT_OPT_PANEL_SPLIT 14
/* Returns 0, -1 for an unknown option, -2 for an invalid value. */
int rbt_set_option(int option, int64_t value);
/* Current value, or -1 for an unknown option. */
int64_t rbt_get_option(int option);

/* Stage timing, for measurement. When enabled, the composite entry points
 * (rbt_solve_ex, rbt_solve_refine, rbt_genp) record a pair of HIP events on
 * their stream around each stage:
 *   0 coefficient draw          work = bytes written
 *   1 two-sided transform       work = algorithmic bytes (read + write of A)
 *   2 one-sided transforms      work = algorithmic bytes
 *   3 diagonal-block factor     work = flops (factor + both inverses)
 *   4 panel block solves        work = flops
 *   5 trailing update GEMM      work = flops, 2 rem^2 kb per launch
 *   6 triangular solves         work = flops
 *   7 residual / norms / Eq. 7  work = bytes of A read
 *   8 pivoted factorization     work = flops 2/3 n^3 (the GEPP re-solve)
 *   9 adjoint outer product     work = bytes of dA written (8 n^2)
 * Disabled by default. Not thread safe. Each timed scope records two events
 * on the stream, a few microseconds of device time apiece: to time one
 * kernel inside a measured run, restrict timing to its stage with
 * RBT_OPT_TIMING_STAGES. */
#define RBT_STAGE_COUNT 10
/* RBT_OPT_TIMING_STAGES: stages timed while timing is enabled, bit s for
 *   stage s (1 .. 2^RBT_STAGE_COUNT - 1; default: all stages). */
#define RBT_OPT_TIMING_STAGES 13
int rbt_timing_enable(int on);

/* Waits for the recorded events and writes, for stages 0..nstages-1, the
 * summed elapsed milliseconds, the number of timed scopes and the summed
 * work (any output pointer may be NULL); then resets the counters. */
int rbt_timing_read(int nstages, double *ms, int64_t *launches, double *work);

#ifdef __cplusplus
}
#endif

#endif /* RBT_H */
