/*
 * seedcg.h -- C ABI of the single-seed Lanczos-CG library for AMD Instinct
 * MI355X (gfx950).
 *
 * The method (Abdel-Rehim, Morgan, Wilcox, "Improved seed methods for
 * symmetric positive definite linear equations with multiple right-hand
 * sides", Sections 1-3) solves A x^j = b^j, j = 1..nrhs, for Hermitian positive
 * definite A in three calls:
 *
 *   sc_seed_lanczos  Lanczos version of CG on right-hand side 1, run for a
 *                    fixed number of steps m (past convergence), with
 *                    periodic reorthogonalization; keeps the basis V and the
 *                    tridiagonal T (Section 3 algorithm, steps 1-9).
 *   sc_project       Galerkin projection of the other right-hand sides over
 *                    the stored basis, X += V T^{-1} V^H R0 (the seeding of
 *                    steps 4 and 7, done in one batched pass).
 *   sc_solve_cg      CG on each seeded system from its projected guess
 *                    (Section 2.2), batched over right-hand sides.
 *
 * Conventions common to every call
 * --------------------------------
 *  - Pointers named *_dev are device pointers (HBM of the current HIP device),
 *    allocated and owned by the caller.  The library never allocates device
 *    memory; scratch space is the caller's `work` buffer, sized by
 *    sc_workspace_size().  Host pointers are named explicitly.
 *  - Vectors are columns: column j of an n-row matrix starts at element j*ld
 *    (ld >= n, counted in elements of the matrix's dtype).  Complex numbers
 *    are interleaved (re, im) pairs.
 *  - Field layout of the Wilson operator (a data format): element
 *    (spin s, colour c, site x) of a spinor column is at index
 *    (s*3 + c)*V + x, V = X*Y*Z*T, x = x0 + X*(x1 + Y*(x2 + Z*x3)).
 *    Links: complex U_mu(x)[a][b] at index ((mu*3 + a)*3 + b)*V + x.
 *    Gamma matrices are Hermitian in the chiral basis with
 *    gamma_5 = diag(1, 1, -1, -1).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; calls that return host results (m_done, iters, relres) synchronise
 *    the stream before returning.
 *  - Every call validates its arguments before touching the device; on an
 *    argument error nothing is written.  Nothing throws or aborts across the
 *    ABI.  Device-detected conditions are reported after the call's sync.
 *    sc_last_error() describes the last failure on the calling thread.
 *  - Calls on one stream are ordered; concurrent calls that share a `work`
 *    buffer race.
 */
#ifndef SEEDCG_H
#define SEEDCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SC_R64 = 0,   /* real double */
    SC_C64 = 1,   /* complex float  (2 x float) */
    SC_C128 = 2,  /* complex double (2 x double) */
    SC_R32 = 3    /* real float */
} sc_dtype;

typedef enum {
    SC_OK = 0,
    SC_NOT_CONVERGED = 1,   /* result usable; some right-hand side above tol at maxit */
    SC_BREAKDOWN = 2,       /* Lanczos found an invariant subspace; *m_done < m, results exact on it */
    SC_ERR_ARG = -1,
    SC_ERR_HIP = -2,
    SC_ERR_NOT_PD = -3,     /* a non-positive LU pivot of T: A is not positive definite */
    SC_ERR_NONFINITE = -4,  /* NaN or Inf met in a norm */
    SC_ERR_WORKSPACE = -5,  /* work buffer smaller than sc_workspace_size() */
    SC_ERR_UNSUPPORTED = -6 /* valid request the library does not implement */
} sc_status;

typedef struct sc_op sc_op;   /* opaque; immutable after creation */

/* ------------------------------------------------------------------ operators
 * The A-apply that drives every step (Section 1: A is real symmetric or
 * complex Hermitian and positive definite).
 */

/* Unscaled 2D five-point Laplacian with zero Dirichlet boundary on an nx-by-ny
 * grid: (A x)_{i,j} = 4 x_{i,j} - x_{i+-1,j} - x_{i,j+-1}.  Vectors: SC_R64
 * (or SC_R32 for the single-precision paths), index i + nx*j.
 * Errors: SC_ERR_ARG if nx or ny < 1 or out is NULL. */
sc_status sc_op_laplace2d(int nx, int ny, sc_op** out);

/* Diagonal A = diag(d) (the matrices of the paper's Examples 1-5).  d_dev:
 * n doubles, positive for an HPD A, owned by the caller and kept alive for the
 * op's lifetime.  Vectors: SC_R64 / SC_R32. */
sc_status sc_op_diag(const double* d_dev, int64_t n, sc_op** out);

/* A = D^H D with the Wilson-Dirac matrix (Section 4 solves the normal
 * equations, two products with D per CG iteration):
 *   (D psi)(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                      + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu) ]
 * dims = {X, Y, Z, T}; periodic in x, y, z; antiperiodic in t when
 * t_antiperiodic != 0.  U64_dev: 4*9*V complex doubles in the link layout
 * above (required).  U32_dev: the same links as complex floats (optional,
 * NULL allowed; needed by the single-precision paths).  Both are held by
 * reference.  Vectors: SC_C128 (or SC_C64), length n = 12*V.
 * Errors: SC_ERR_ARG on a dimension < 1, a NULL U64_dev, or kappa not finite. */
sc_status sc_op_wilson_normal(const int dims[4], const void* U64_dev, const void* U32_dev,
                              double kappa, int t_antiperiodic, sc_op** out);

/* Q = gamma_5 D, gamma_5 = diag(1, 1, -1, -1) in spin (the chiral basis):
 * Hermitian and indefinite, one product with D per apply (Section 4 names it
 * as the alternative to D^H D).  The system D x = b is Q x = gamma_5 b.
 * Arguments, layouts and errors as sc_op_wilson_normal.  Used by
 * sc_indefinite_solve and sc_solve_minres; with sc_seed_lanczos it turns
 * the positive-pivot check off and forms x^1 as the minimum residual over the
 * basis (QR of the (m+1) x m tridiagonal matrix) instead of by the LU. */
sc_status sc_op_wilson_g5(const int dims[4], const void* U64_dev, const void* U32_dev, double kappa,
                          int t_antiperiodic, sc_op** out);

/* Checks on the GPU whether every link of a Wilson operator (either kind) is
 * in SU(3): the largest over the links of the entrywise moduli of
 * U U^H - 1 and of |det U - 1|, in FP64 from U64_dev, is returned in
 * *deviation (host, may be NULL; +inf if a link holds a value that is not
 * finite).  When it is at most 1e-9 and the op has U32_dev, the op's
 * single-precision passes from then on read rows 0 and 1 of each link and
 * rebuild row 2 as the complex conjugate of their cross product (which holds
 * for unitary matrices of determinant 1): 12 instead of 18 reals per link,
 * equal to the stored row up to FP32 rounding.  *rebuild (host, may be NULL)
 * is 1 then and 0 otherwise, and 0 until this is called.  The links must not
 * change afterwards to values outside SU(3) unless this is called again.
 * Not part of the method: a smaller form of the data it reads.  Runs on
 * `stream`, allocates at most 8 KB of device memory for the duration of the call
 * and synchronizes the stream once; it changes the op, so no other call may
 * use the op meanwhile.  Errors: SC_ERR_ARG for an op that is not a Wilson
 * operator; SC_ERR_HIP. */
sc_status sc_op_wilson_check_su3(sc_op* op, void* stream, double* deviation, int* rebuild);

sc_status sc_op_destroy(sc_op* op);

/* Vector length n and the op's full-precision dtype (SC_R64 or SC_C128). */
sc_status sc_op_info(const sc_op* op, int64_t* n, sc_dtype* dtype);

/* Y = A X for k columns.  dtype is the op's dtype or its single-precision
 * counterpart (SC_R32 / SC_C64; Wilson needs U32_dev).  Needs
 * sc_workspace_size(op, SC_CALL_APPLY, k, 0, dtype) bytes of work. */
sc_status sc_op_apply(const sc_op* op, sc_dtype dtype, const void* X_dev, int64_t ldx,
                      void* Y_dev, int64_t ldy, int k, void* work_dev, size_t work_bytes,
                      void* stream);

/* One Wilson stencil pass for k columns (no workspace):
 * which = 0: Y = D X, 1: Y = D^H X, 2: Y = H X, 3: Y = H^H X,
 * where D = 1 - kappa H (H, the hopping term, gives dD/dkappa = -H).
 * Errors: SC_ERR_ARG for a non-Wilson op or which outside 0..3. */
sc_status sc_wilson_dslash(const sc_op* op, sc_dtype dtype, int which, const void* X_dev,
                           int64_t ldx, void* Y_dev, int64_t ldy, int k, void* stream);

/* Launch shape of the Wilson stencil chosen by the library's autotuner for
 * this lattice, precision and column count k (not part of the method).  The
 * first pass with a new (lattice, dtype, k) times each candidate shape on the
 * caller's buffers, which adds one host synchronisation to that call, and
 * keeps the fastest; SEEDCG_TUNE=0 in the environment selects fixed defaults,
 * and no tuning happens while the stream is being captured.
 * variant (host) = order * 16 + shape * 4 + chunk, -1 if not tuned yet.
 * shape 0: hops unrolled, 1 column per thread; 1, 2, 3: rolled hop loop with
 * 1, 2, 4 columns per thread (FP64: 2 for shape 3).  The (256-site tile,
 * column group) work items are enumerated in chunks of G column groups, the G
 * groups of a tile consecutive: chunk 0: G = all groups (a tile's columns
 * together), 1: G = 1 (one group sweeps the lattice before the next), 2: G =
 * 2, 3: G = 4.  order 0: tiles in site order; 1: blocks of 4 tiles along z
 * taken through all time slices before the next block (only when each time
 * slice holds a multiple of 4 whole tiles, else as order 0).  32..43: for
 * lattices with X Y = 256 only, one block per xy-plane walking t through
 * segments of 4, 8, 16 time slices, x and y neighbours staged in LDS, t
 * neighbours kept in registers: 32 + 6 * o + 3 * (c - 1) + {0, 1, 2} for
 * segments of {4, 8, 16}, c = 1 or 2 columns per thread (2: FP32 only, FP64
 * uses 1), o = 0: the planes of a segment are consecutive work items, 1: the
 * column groups of a plane are.  44: one wave per direction mu and 64
 * sites, the four partial sums added in LDS (for few columns).  45..56 and
 * 57..68: the t-march shapes of 32..43 (numbered alike from 45 and 57) with
 * blocks of 2 and 4 consecutive z-planes, whose z neighbours inside the
 * block are staged in LDS too; where the planes do not fit LDS (4 planes of
 * 2 columns, FP64 beyond 2 planes) or do not divide Z, the launch uses the
 * next smaller plane count.  69..86: FP32 D and D^H passes on lattices with
 * X = Y = 16 (and |kappa| >= 1e-6), for k > 1: one block per xy-plane and
 * column group marching t, x neighbours exchanged between lanes (DPP), y
 * neighbours through LDS as half spinors already multiplied by the source
 * site's link; 69 + 6 * (c - 1) + 3 * o + {0, 1, 2} for c = 1, 2 columns
 * per thread, segments of {4, 8, 16} slices, o = 0: the planes of a segment
 * are consecutive work items, 1: the column groups of a plane are;
 * 81 + 3 * (c - 1) + {0, 1, 2}: quads of 4 consecutive planes (2 or 1 when
 * Z is not a multiple of 4), the planes of one column group consecutive,
 * then the next group on the same quad.
 * us (host, SC_WILSON_VARIANTS floats): measured microseconds per pass of each
 * candidate (-1 if not run). */
#define SC_WILSON_VARIANTS 87
sc_status sc_wilson_tune_info(const sc_op* op, sc_dtype dtype, int k, int* variant, float* us);

/* Pin the stencil launch shape for (this op's lattice, dtype, k) instead of
 * tuning it (variant as above); variant -1 forgets the choice so the next
 * pass tunes again.  Errors: SC_ERR_ARG for a non-Wilson op, k < 1, a
 * variant outside -1..SC_WILSON_VARIANTS-1, or a t-march variant (32..43,
 * 45..68) on a lattice with X Y != 256. */
sc_status sc_wilson_tune_set(const sc_op* op, sc_dtype dtype, int k, int variant);

/* Host-only check of the addressing of the DPP-form stencil shapes (69..86),
 * whose loads and stores go through buffer descriptors: an access outside
 * its descriptor's record would read zero or be dropped instead of faulting.
 * Walks, on the CPU and with the kernel's own index functions, every access
 * that one pass over a lattice of dims[4] = {X, Y, Z, T} with k columns of
 * leading dimensions ldx (source) and ldy (destination; complex elements)
 * would make, and counts those outside their record (*outside) among all
 * checked (*accesses); a correct shape gives *outside = 0.  Touches no GPU.
 * Errors: SC_ERR_ARG for a variant that is not a DPP-form shape, or a
 * lattice it does not run on (X = Y = 16, 288 V < 2^31 bytes). */
sc_status sc_wilson_range_check(const int* dims, int variant, int k, int64_t ldx, int64_t ldy, int64_t* accesses,
                                int64_t* outside);

/* ------------------------------------------------------------------ workspace */
typedef enum {
    SC_CALL_APPLY = 0,
    SC_CALL_SEED = 1,
    SC_CALL_PROJECT = 2,
    SC_CALL_CG = 3,
    SC_CALL_KAPPA_GRAD = 4,
    SC_CALL_RELATED = 5,
    SC_CALL_MULTISEED = 6,
    SC_CALL_SEEDED = 7,
    SC_CALL_MINRES = 8,
    SC_CALL_INDEFINITE = 9
} sc_call;

/* Bytes of `work` needed by a call.  k: right-hand sides per call (a call
 * with more columns than the k it was sized for needs a new query); m: basis
 * size (seed, project); dtype: vector dtype of the call (for SC_CALL_CG pass
 * the op dtype and set k; the mixed-precision solver needs the same query with
 * the single-precision dtype).  For SC_CALL_PROJECT op may be NULL when n is
 * passed through *bytes on entry (in: n, out: bytes). */
sc_status sc_workspace_size(const sc_op* op, int call, int k, int m, sc_dtype dtype, size_t* bytes);

/* ------------------------------------------------------------------ seed phase
 * Lanczos version of CG on right-hand side 1 (Section 3 algorithm, steps 1-9),
 * run for exactly m steps, with the readings:
 *   - alpha_i = Re(v_i^H f); T_m is real symmetric tridiagonal;
 *   - step 8 (when i is a multiple of reorth_freq, i >= 2; 0 = never,
 *     1 = every step) is one pass of classical Gram-Schmidt: v_i and f
 *     against v_1..v_{i-1}, renormalise v_i, then f against the new v_i;
 *     alpha and beta keep their recurrence values;
 *   - breakdown when beta_i <= 1e-12 * max_k |alpha_k|.
 * b1_dev: right-hand side 1 in the op dtype.  x1_dev (op dtype): in, the
 * initial guess (zeros allowed); out, x0 + V_m T_m^{-1} (beta_0 e_1), the
 * Lanczos-CG iterate after m_done steps.
 * V_dev: n x (m+1) basis, column i-1 = v_i, leading dimension ldv >= n, dtype
 * v_dtype: the op dtype (all-FP64 arithmetic) or its single-precision
 * counterpart (FP32 vectors and storage; FP64 dot products, recurrences and
 * reorthogonalization sums).
 * alpha_dev: m doubles (alpha_1..alpha_m); beta_dev: m+1 doubles
 * (beta_0..beta_m).  m_done (host): steps completed.
 * Returns SC_OK, SC_BREAKDOWN (m_done < m), SC_ERR_NOT_PD (m_done = the last
 * step with a positive pivot), SC_ERR_NONFINITE, or an argument/HIP error.
 * Synchronises `stream` once, at the end. */
sc_status sc_seed_lanczos(const sc_op* op, const void* b1_dev, void* x1_dev, int m, int reorth_freq,
                          void* V_dev, int64_t ldv, sc_dtype v_dtype, double* alpha_dev,
                          double* beta_dev, int* m_done, void* work_dev, size_t work_bytes,
                          void* stream);

/* ------------------------------------------------------------------ projection
 * X += V_m T_m^{-1} V_m^H R0 for k columns: the Galerkin projection over the
 * stored basis that seeds right-hand sides 2..nrhs (steps 4 and 7 in batched
 * form).  T_m has diagonal alpha_1..alpha_m and off-diagonal beta_1..beta_{m-1}
 * and is solved with the LU recurrences of step 6 (no pivoting).
 * V_dev: n x m, ldv, v_dtype (SC_C128/SC_C64 or SC_R64/SC_R32).
 * R0_dev, X_dev: n x k in vec_dtype (SC_C128 or SC_R64; the full-precision
 * type matching V).  Sums are accumulated in FP64.  Asynchronous.  For the
 * basis of an indefinite op the LU of T_m need not exist: sc_indefinite_solve
 * forms minimum-residual guesses through the (m+1) x m matrix instead. */
sc_status sc_project(int64_t n, const void* V_dev, int64_t ldv, sc_dtype v_dtype, int m,
                     const double* alpha_dev, const double* beta_dev, sc_dtype vec_dtype,
                     const void* R0_dev, int64_t ldr, int k, void* X_dev, int64_t ldx,
                     void* work_dev, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ projection, no allocation
 * sc_project without a work buffer, for callers that cannot allocate device
 * memory: code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, layouts, result and errors as
 * sc_project, minus work_dev/work_bytes.  The scratch space (the m x k
 * coefficient block, the contraction's partial sums, the tridiagonal solve's
 * work) lives in an array of SC_NOALLOC_SCRATCH_BYTES bytes of device memory
 * that the library holds on every GPU it runs on until the process ends; the
 * call itself allocates nothing.  Sizes whose scratch
 * (sc_workspace_size(NULL, SC_CALL_PROJECT, k, m, ...) with n passed in) would
 * exceed it are rejected with SC_ERR_WORKSPACE before anything is launched.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * device (two streams, two threads) race.  The optional benchmark timer never
 * times this call. */
#define SC_NOALLOC_SCRATCH_BYTES (64u << 20)
sc_status sc_project_noalloc(int64_t n, const void* V_dev, int64_t ldv, sc_dtype v_dtype, int m,
                             const double* alpha_dev, const double* beta_dev, sc_dtype vec_dtype,
                             const void* R0_dev, int64_t ldr, int k, void* X_dev, int64_t ldx, void* stream);

/* ------------------------------------------------------------------ CG
 * Plain CG (Hestenes-Stiefel) on each of k columns, batched: B_dev and X_dev
 * (in: guesses, out: solutions) are n x k in the op dtype.  Stops each column
 * when its recursively updated residual satisfies ||r|| <= tol ||b||, then
 * recomputes the true residual and restarts from it (at most 5 times) while
 * it is above tol.  One iteration = one A-apply.
 * mixed = 0: FP64 throughout.  mixed = 1: FP32 vectors and operator with FP64
 * reliable updates: x and the true residual b - A x are kept in FP64 and
 * recomputed whenever the FP32 residual has fallen by 1e4x since the last
 * update, and at FP32 convergence; a column is converged only when its FP64
 * true residual is <= tol.  (Wilson needs U32_dev.)
 * iters (host, k ints), relres (host, k doubles: true relative residuals).
 * Returns SC_OK or SC_NOT_CONVERGED.  Synchronises once per chunk of
 * iterations. */
sc_status sc_solve_cg(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev,
                      int64_t ldx, int k, double tol, int maxit, int* iters, double* relres,
                      void* work_dev, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ the single-seed method as one call
 * The seed algorithm of Section 3 (steps 1-9) on system 1 (column 0 of B)
 * from x = 0, m Lanczos steps with reorthogonalization every reorth_freq
 * (0: never; the basis is complex64 / FP32 when mixed = 1); columns 1..k-1
 * seeded by the projection over its basis (steps 4 and 7, batched:
 * x^j = V_m T_m^{-1} V_m^H b^j); then CG (Section 2.2, as sc_solve_cg with the
 * same mixed) finishes every column from its guess.  The result is that of
 * sc_seed_lanczos, sc_project and sc_solve_cg called in turn from zero
 * guesses (up to rounding order); here x^1 and the other guesses are formed
 * in one pass over the basis.  The basis is not returned.
 *   B_dev: n x k (ldb), the op's dtype, read only.  X_dev: n x k (ldx),
 *   written.  iters (host, k): A-applies per system (system 1 counts its m_done
 *   seed steps).  relres (host, k): true relative residuals.  m_done (host).
 * Needs sc_workspace_size(op, SC_CALL_SEEDED, k, m, dtype) bytes (dtype: the
 * op's dtype, or its single-precision dtype when mixed = 1).  Synchronises
 * the host once after the seed phase and once per chunk of CG iterations.
 * Returns SC_OK, SC_NOT_CONVERGED, SC_BREAKDOWN (seed phase stopped early at
 * an invariant subspace), or an error (SC_ERR_NOT_PD, SC_ERR_NONFINITE from
 * the seed phase; SC_ERR_ARG, SC_ERR_WORKSPACE, SC_ERR_HIP). */
sc_status sc_seeded_solve(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev,
                          int64_t ldx, int k, int m, int reorth_freq, double tol, int maxit, int* iters,
                          double* relres, int* m_done, void* work_dev, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ MINRES (Hermitian indefinite)
 * MINRES (Paige and Saunders) on the k columns of B from the guesses in X,
 * FP64, per-column scalars on the device: the finishing solver of the
 * indefinite variant (for any Hermitian op; Q = gamma_5 D in particular).
 * Stops a column when its recursive residual norm is <= tol ||b||, then
 * verifies the true residual and restarts from r = b - A x while it is above
 * tol (at most 5 times, as sc_solve_cg).  Synchronises once per 8
 * iterations.  B_dev, X_dev (in/out): n x k in the op's dtype (ldb, ldx).
 * iters (host, k): A-applies in the iterations; relres (host, k): true
 * relative residuals.  Needs sc_workspace_size(op, SC_CALL_MINRES, k, 0,
 * op dtype) bytes.  Returns SC_OK or SC_NOT_CONVERGED, or an error. */
sc_status sc_solve_minres(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx,
                          int k, double tol, int maxit, int* iters, double* relres, void* work_dev,
                          size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ the indefinite variant
 * The seed method for a Hermitian indefinite op (Q = gamma_5 D; the remark of
 * Section 3 on indefinite systems: a QR factorization of the Lanczos
 * tridiagonal matrix in place of its LU), FP64, from zero guesses:
 *   1. the Lanczos steps of the seed algorithm (1, 2, 5, 8, 9; m steps,
 *      reorthogonalization every reorth_freq) on column 0 of B;
 *   2. every column's guess x^j = V_m y_j, y_j = argmin || c_j - T~_m y || with
 *      T~_m the (m+1) x m tridiagonal matrix, c_j = V_{m+1}^H b^j (c_1 =
 *      beta_0 e_1), by a QR factorization of T~_m: the minimum residual over
 *      the basis;
 *   3. MINRES (as sc_solve_minres) from the guesses.
 * B_dev: n x k (ldb), read only; X_dev: n x k (ldx), written.  iters (host,
 * k): A-applies (column 0 counts its m_done seed steps); relres (host, k);
 * m_done (host).  Needs sc_workspace_size(op, SC_CALL_INDEFINITE, k, m, op
 * dtype) bytes.  Returns SC_OK, SC_NOT_CONVERGED, SC_BREAKDOWN (the seed
 * phase met an invariant subspace), or an error. */
sc_status sc_indefinite_solve(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx,
                              int k, int m, int reorth_freq, double tol, int maxit, int* iters,
                              double* relres, int* m_done, void* work_dev, size_t work_bytes,
                              void* stream);

/* ------------------------------------------------------------------ related right-hand sides
 * Single seeding of related systems (Section 2.3, the algorithm for related
 * right-hand sides, steps 1-4; Example 3).  System 1 (column 0 of B) is seeded
 * by the Lanczos phase (m steps, reorthogonalization every reorth_freq; the
 * basis is complex64 / FP32 when mixed = 1) from X = 0 and finished with CG;
 * columns 1..k-1 are projected over its basis and their residuals r^i = b^i -
 * A x^i are formed once.  Then the systems are solved in column order by CG
 * from their carried guesses, and after system j converges its CG correction
 * x_cg = x^j - x^j_bcg (x^j_bcg: its guess before CG; zero for system 1)
 * seeds every later system i: delta = (x_cg^H r^i) / (x_cg^H r^j_bcg),
 * x^i += delta x_cg, r^i -= delta r^j_bcg (r^j_bcg: the residual system j
 * started CG from; delta = 0 when the denominator is 0).
 *   B_dev: n x k (ldb), the op's dtype, read only.  X_dev: n x k (ldx),
 *   written.  iters (host, k): A-applies per system (system 1 counts its m_done
 *   seed steps).  relres (host, k): true relative residuals.  m_done (host).
 * Needs sc_workspace_size(op, SC_CALL_RELATED, k, m, dtype) bytes (dtype: the
 * op's dtype, or its single-precision dtype when mixed = 1).  Returns SC_OK,
 * SC_NOT_CONVERGED, SC_BREAKDOWN (seed phase stopped early), or an error. */
sc_status sc_related_solve(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev,
                           int64_t ldx, int k, int m, int reorth_freq, double tol, int maxit, int* iters,
                           double* relres, int* m_done, void* work_dev, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ multiple seeding (comparator)
 * Standard seed CG, the method the paper compares single seeding against
 * (Section 2.1, after Chan and Wan; Example 1, Table 2.1).  The k systems
 * (columns of B) are solved in order by CG from X = 0; while system j
 * iterates, every later system i is projected over each new A-conjugate
 * direction p (q = A p): c = (p^H r^i) / (p^H q), x^i += c p, r^i -= c q, with
 * r^i the carried residual of system i.  System j then starts its own CG from
 * that guess with its true residual.  FP64 in the op's dtype; two host
 * synchronisations per iteration (a comparator, not a fast path).
 *   B_dev: n x k (ldb), read only.  X_dev: n x k (ldx), written.  iters (host,
 *   k): CG iterations (A-applies) of each system's own solve.  relres (host, k):
 *   true relative residuals.
 * Needs sc_workspace_size(op, SC_CALL_MULTISEED, k, 0, dtype) bytes.  Returns
 * SC_OK, SC_NOT_CONVERGED, SC_ERR_NOT_PD (p^H A p <= 0) or an argument error. */
sc_status sc_multiple_seed_solve(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx,
                                 int k, double tol, int maxit, int* iters, double* relres, void* work_dev,
                                 size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ timing
 * Optional event timing of the library's main kernels, for benchmarks (not
 * part of the method).  sc_timer_enable(every) with every >= 1 clears earlier
 * records and, from then on, brackets one launch in `every` of each stencil
 * class below (a fixed pseudo-random sample; every = 1 times all of them) and
 * every launch of classes 2 and 3 with two HIP events on the launch's own
 * stream, recording that launch's algorithmic bytes and flops;
 * sc_timer_enable(0) stops recording.  Launches inside a
 * stream capture are never timed.  sc_timer_read(cls, ...) waits for the
 * recorded events and returns, for class cls, the summed kernel time (ms),
 * the number of timed launches and their summed algorithmic bytes and flops:
 *   0  Wilson stencil pass, FP32, k = 1: (48k + 72)*4 bytes and 1368k (D,
 *      D^H) or 1320k (H, H^H) flops per site for k columns;
 *   1  Wilson stencil pass, FP64, k = 1: (48k + 72)*8 bytes per site, same flops;
 *   2  G = V^H W: V, W read once, G written; 8 n M N flops (complex);
 *   3  X += V Y:  V read once, X read and written; 8 n M N flops (complex);
 *   4  Wilson stencil pass, FP32, k > 1 (bytes and flops as class 0);
 *   5  Wilson stencil pass, FP64, k > 1 (bytes and flops as class 1).
 * Errors: SC_ERR_ARG for an unknown class or a NULL pointer. */
sc_status sc_timer_enable(int every);
sc_status sc_timer_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops);

/* ------------------------------------------------------------------ batches
 * Several independent systems, each single-seeded, advanced together: the
 * seed phases of all systems (static control flow) are captured in one HIP
 * graph on forked streams and launched once, so every lattice's Lanczos steps
 * run concurrently; the graph is cached and replayed when the same argument
 * set is solved again.  Then each system is projected and finished with CG on
 * its own stream, concurrently.  Per system: X = 0 initially, RHS 1 seeds
 * (m steps, reorthogonalization every reorth_freq), columns 2..k are projected
 * over its basis, all k columns finish with CG to tol (mixed = 1: complex64
 * basis, FP32 bulk, FP64 reliable updates and scalars).  The library fills
 * m_done and status (an sc_status) of each system; iters and relres are host
 * arrays of k entries.  All device buffers, including `work`
 * (sc_batch_workspace_size bytes), are the caller's.  The call synchronises
 * `stream` and returns SC_OK, SC_NOT_CONVERGED or SC_BREAKDOWN if every system
 * did, else the first error. */
typedef struct {
    const sc_op* op;
    const void* B_dev;   /* n x k, op dtype */
    int64_t ldb;
    void* X_dev;         /* n x k, op dtype (output) */
    int64_t ldx;
    int k;
    int m;
    int reorth_freq;
    double tol;
    int maxit;
    int mixed;
    int* iters;          /* host, k */
    double* relres;      /* host, k */
    int m_done;          /* out */
    int status;          /* out */
} sc_batch_system;

sc_status sc_batch_workspace_size(int nsys, const sc_batch_system* systems, size_t* bytes);
sc_status sc_batch_solve(int nsys, sc_batch_system* systems, void* work_dev, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ gradient
 * Derivative with respect to kappa of L = sum_j Re<eta_j, x_j>, where
 * x_j = A^{-1} b_j solves the Wilson normal equations (not part of the paper's
 * method: it lets the seeded solve sit inside a differentiable program).  Given
 * the solutions X and the adjoint solutions L (lambda_j = A^{-1} eta_j, which
 * the caller obtains with sc_project / sc_solve_cg seeded from the forward
 * basis), writes to *grad (host)
 *   sum_j Re[(H lambda_j)^H (D x_j) + (D lambda_j)^H (H x_j)],
 * since dA/dkappa = -(H^H D + D^H H) for D = 1 - kappa H.  X_dev, L_dev: n x k
 * complex doubles.  Needs sc_workspace_size(op, SC_CALL_KAPPA_GRAD, k, 0, ...)
 * bytes of work.  Synchronises the stream.  Errors: SC_ERR_ARG for a
 * non-Wilson op or bad pointers, SC_ERR_WORKSPACE. */
sc_status sc_wilson_kappa_grad(const sc_op* op, const void* X_dev, int64_t ldx, const void* L_dev,
                               int64_t ldl, int k, double* grad, void* work_dev, size_t work_bytes,
                               void* stream);

/* Description of the last failure on the calling thread (valid until the next
 * call on that thread); "" when the last call succeeded. */
const char* sc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEEDCG_H */
