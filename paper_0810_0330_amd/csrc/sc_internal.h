// Internal declarations: the operator object and the launchers shared by the
// host drivers.
#pragma once

#include <memory>

#include "sc_common.h"

enum sc_op_kind { SC_OPK_LAPLACE2D = 0, SC_OPK_DIAG = 1, SC_OPK_WILSON = 2, SC_OPK_WILSON_G5 = 3 };

struct sc_op {
    int kind;
    int64_t n;          // vector length in elements of `dtype`
    sc_dtype dtype;     // SC_R64 or SC_C128
    // Laplacian
    int nx = 0, ny = 0;
    // diagonal
    const double* d = nullptr;
    // Wilson
    int dims[4] = {0, 0, 0, 0};  // X, Y, Z, T
    int64_t vol = 0;
    const void* U64 = nullptr;
    const void* U32 = nullptr;
    double kappa = 0.0;
    int antiperiodic = 1;
    // every link of U64 is in SU(3) to within 1e-9 (checked at creation): the
    // single-precision passes read rows 0 and 1 of a link and rebuild row 2
    int su3 = 0;
    // distinct for every op the process creates (an op allocated at a freed
    // op's address is still a different op to the caches keyed on it)
    uint64_t gen = 0;
};

// operators built on the Wilson links (D^H D, and gamma_5 D, which is Hermitian indefinite)
inline bool has_links(const sc_op* op) { return op->kind == SC_OPK_WILSON || op->kind == SC_OPK_WILSON_G5; }

namespace sc {

// Column pointer list for the tall-skinny kernels (up to kMaxCols columns).
constexpr int kMaxCols = 32;
template <typename T>
struct ColPtrs {
    T* p[kMaxCols];
};

// ---------------------------------------------------------------- stencils (k_stencil.hip)
// Y = A X for k columns, all arrays in the precision selected by `single`
// (ld in elements of that dtype).  tmp: k*n elements (Wilson only).
sc_status op_apply(const sc_op* op, bool single, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                   void* tmp, hipStream_t s);
// elements of scratch op_apply needs per column
int64_t op_apply_tmp_elems(const sc_op* op);

// Per-column state of the batched CG (cg.hip), read by the fused stencil epilogue.
struct CGCol {
    double rho;      // ||r||^2 of the current recurrence
    double rho_prev; // rho of the previous iteration
    double beta;     // rho / rho_prev
    double bnorm2;   // ||b||^2
    double tol2;     // tol^2 ||b||^2
    double rmax2;    // largest ||r||^2 since the last reliable update
    int active;      // iterating
    int iters;       // A-applies inside the loop so far
    int maxit;
    int flag;        // 1: recursive residual at tol; 2: mixed, reliable update due
};

// One CG iteration's operator work for the Wilson normal operator, fused,
// when the tuned stencil shape for (lattice, precision, k) is a t-march one:
// tmp = D p with partials of ||D p_j||^2 = <p_j, A p_j> in part_pq, then the
// D^H pass, whose epilogue applies r_j -= alpha_j (A p_j) with alpha_j =
// rho_j / <p_j, A p_j> for the active columns of st and leaves partials of
// ||r_j||^2 in part_rr (A p is not stored).  *G = partials per column (both
// arrays, index j * G + i), or 0 when the fused form does not apply (nothing
// was launched).
sc_status wilson_cg_fused(const sc_op* op, bool single, const void* p, void* tmp, int k, const CGCol* st,
                          double* part_pq, void* r, int64_t ldr, double* part_rr, int max_parts, int* G,
                          hipStream_t s);
// Y = A X; for the Wilson normal operator, when the tuned D-pass shape can, it
// also leaves per-column partial sums of ||D x_j||^2 = <x_j, A x_j> in
// part[j * G + i] (i < G <= max_parts) and sets G; otherwise G = 0.
sc_status op_apply_norm(const sc_op* op, bool single, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                        void* tmp, double* part, int max_parts, int* G, hipStream_t s);
// one Wilson pass: which 0 = D, 1 = D^H, 2 = H, 3 = H^H
sc_status wilson_pass(const sc_op* op, bool single, int which, const void* X, int64_t ldx, void* Y, int64_t ldy,
                      int k, hipStream_t s);

// autotuned stencil launch shape for (op lattice, precision, k): variant id
// (-1 if not tuned yet) and the measured microseconds of each candidate
sc_status wilson_tune_query(const sc_op* op, bool single, int k, int* variant, float* us);
// SU(3) check of a Wilson operator's links (links.hip): sets op->su3 when every
// link of U64 is in SU(3) to within kSu3Tol and the op has U32
constexpr double kSu3Tol = 1e-9;
sc_status wilson_check_su3(sc_op* op, hipStream_t s, double* deviation, int* rebuild);
// pin a variant for (lattice, precision, k); variant < 0 forgets the choice
sc_status wilson_tune_pin(const sc_op* op, bool single, int k, int variant);
// host-side walk of every buffer access of a DPP-form stencil launch (no GPU)
sc_status wilson_tx_check(const int dims[4], int v, int k, int64_t ldx, int64_t ldy, int64_t* accesses,
                          int64_t* outside);

// ---------------------------------------------------------------- streaming kernels (k_blas.hip)
// All act on "real views": a complex column of n elements is 2n reals.
// z = a*x + b*y  (y may be null when b == 0); types: 0 = double, 1 = float
sc_status lincomb(int zt, void* z, int64_t ldz, int xt, const void* x, int64_t ldx, int yt, const void* y,
                  int64_t ldy, int64_t N, int k, double a, double b, hipStream_t s);
// res[j] = sum_i x[i,j]*y[i,j] (FP64 accumulation), deterministic split reduction.
// part: k*kMaxRedBlocks doubles, ctr: k zeroed counters.
sc_status dot(int xt, const void* x, int64_t ldx, int yt, const void* y, int64_t ldy, int64_t N, int k,
              double* res, double* part, unsigned* ctr, hipStream_t s);
template <typename T>
sc_status fill(T* p, int64_t n, T v, hipStream_t s);
// res[b] = sum of part[b*G .. b*G+G) (one block per column), fixed order
__global__ void k_dot_finish(const double* part, int G, double* res);

// ---------------------------------------------------------------- tall-skinny (k_tsgemm.hip)
// G[a*N + j] = sum_r conj(V[r,a]) W_j[r]  (a < M, j < N <= kMaxCols); G complex or real FP64.
// part: gemm_cn_part_elems(n, M, N) doubles.
size_t gemm_cn_part_doubles(int64_t n, int M, int N, bool cplx);
sc_status gemm_cn(bool cplx, bool vsingle, const void* V, int64_t ldv, int64_t n, int M, bool wsingle,
                  const ColPtrs<const void>& W, int N, double* G, double* part, const int* halt, hipStream_t s);
// X_j[r] += scale * sum_a V[r,a] Y[a*N + j]
sc_status gemm_nn(bool cplx, bool vsingle, const void* V, int64_t ldv, int64_t n, int M, const double* Y, int N,
                  bool xsingle, const ColPtrs<void>& X, double scale, const int* halt, hipStream_t s);
// least squares with the (M+1) x M tridiagonal matrix (QR); C is M+1 x N, y in its first M rows; work 5 M doubles
sc_status tridiag_lsq(const double* alpha, const double* beta, int M, double* C, int N, bool cplx, double* work,
                      hipStream_t s);
// Y (M x N, complex or real, row-major [a*N+j]) <- T_M^{-1} Y by the LU recurrences.
// If e1_beta0 != null, Y is first set to beta0 e_1 (N = 1).  work: 2*M doubles.
sc_status tridiag_solve(const double* alpha, const double* beta, int M, double* Y, int N, bool cplx,
                        const double* e1_beta0, double* work, const int* halt, hipStream_t s);

// ---------------------------------------------------------------- seed phase (seed.hip)
struct SeedState;
struct SeedWork {
    void* av;        // A v_i          (vector precision)
    void* f;         // f              (vector precision)
    void* tmp;       // op scratch     (vector precision)
    double* r64;     // r0^1           (FP64)
    double* ax64;    // A x0           (FP64)
    void* tmp64;     // op scratch     (FP64)
    double* part_a;  // partials of alpha_i
    double* part_f;  // partials of ||f||^2
    double* part_v;  // partials of ||v_i||^2 (reorthogonalization)
    double* delta;   // LU pivots delta_1..delta_m (index i)
    SeedState* st;
    double* G;       // reorthogonalization coefficients, (m) x 2 complex
    double* G2;      // one complex coefficient
    double* gpart;   // gemm_cn partials
    double* y;       // T^{-1} beta_0 e_1 (m + 1 complex; the least-squares right-hand side for an indefinite op)
    double* trid;    // LU work (2m), or QR work (5m) for an indefinite op
};
size_t seed_workspace(const sc_op* op, int m, bool single);
SeedWork seed_carve(void* work, size_t work_bytes, const sc_op* op, int m, bool single, bool* ok);
sc_status seed_pretune(const sc_op* op, bool single, const SeedWork& w, hipStream_t s);
// steps 1-9 enqueued with no host synchronisation (capturable)
// indef: no positive-pivot check (always so for gamma_5 D)
sc_status seed_enqueue_any(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv,
                           sc_dtype vdt, double* alpha, double* beta, const SeedWork& w, hipStream_t s,
                           bool indef = false);
// one synchronisation: final state, then x^1 (unless form_x1 is false)
sc_status seed_finalize_any(const sc_op* op, void* x1, void* V, int64_t ldv, sc_dtype vdt, double* alpha,
                            double* beta, int* m_done, const SeedWork& w, hipStream_t s, sc_status* result,
                            bool form_x1 = true);

// ---------------------------------------------------------------- projection and CG
// bytes of work of project_impl for k right-hand sides (any k up to kMaxCols needs the same)
size_t project_workspace(int64_t n, int m, int k, bool cpl);
sc_status project_impl(int64_t n, const void* V, int64_t ldv, sc_dtype vdt, int m, const double* alpha,
                       const double* beta, sc_dtype xdt, const void* R0, int64_t ldr, int k, void* X, int64_t ldx,
                       void* work, size_t work_bytes, hipStream_t s);
size_t cg_workspace(const sc_op* op, int k, bool mixed);
// The batched CG of solve_cg as a steppable object (cg.hip): start() forms the
// residuals and column states (one host synchronisation); iterate(n) enqueues
// n iterations and nothing else, so a fixed n can be captured into a graph;
// check() reads the column states, applies the stall rules and makes the due
// reliable updates; verify() checks every column's true residual once none is
// active and restarts those above tol (again = true).  state_index() is the
// copy of the double-buffered column state the next iteration reads (an even
// number of iterations returns to it).
class CGRun {
   public:
    virtual ~CGRun() = default;
    virtual sc_status start() = 0;
    virtual bool any_active() const = 0;
    virtual int chunk() const = 0;
    virtual int state_index() const = 0;
    virtual hipStream_t stream() const = 0;
    virtual sc_status iterate(int n) = 0;
    virtual sc_status check(bool* any) = 0;
    virtual sc_status verify(bool* again) = 0;
    virtual void results(int* iters, double* relres, sc_status* result) const = 0;
};
// the CG of solve_cg on the caller's work buffer (null and *st set on error)
std::unique_ptr<CGRun> cg_make(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k,
                               double tol, int maxit, void* work, size_t work_bytes, hipStream_t s, sc_status* st);
// one k-column pass through the CG workspace, so that the stencil shape of the
// CG passes is tuned now (e.g. before systems start running concurrently)
sc_status cg_pretune(const sc_op* op, int mixed, int k, void* work, size_t work_bytes, hipStream_t s);
sc_status solve_cg(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                   int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s);

// ---------------------------------------------------------------- batches (batch.hip)
// drop every cached batch graph that was recorded for this op (called when the op is destroyed)
void batch_forget_op(const sc_op* op);
// seed_enqueue_any replayed from a cached graph (batch.hip); for small systems,
// whose seed phase is a chain of short launches
sc_status seed_enqueue_cached(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv,
                              sc_dtype vdt, double* alpha, double* beta, const SeedWork& w, hipStream_t s,
                              bool single);

// ---------------------------------------------------------------- multiple seeding (multiseed.hip)
size_t multiseed_workspace(const sc_op* op, int k);
sc_status multiseed_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                          int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s);

// ---------------------------------------------------------------- MINRES and the indefinite variant
size_t minres_workspace(const sc_op* op, int k);
sc_status minres_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                       int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s);
size_t indefinite_workspace(const sc_op* op, int k, int m);
sc_status indefinite_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m, int freq,
                           double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                           size_t work_bytes, hipStream_t s);

// ---------------------------------------------------------------- the single-seed method as one call (seeded.hip)
size_t seeded_workspace(const sc_op* op, int k, int m, bool mixed);
sc_status seeded_solve(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m,
                       int freq, double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                       size_t work_bytes, hipStream_t s);

// ---------------------------------------------------------------- related right-hand sides (related.hip)
size_t related_workspace(const sc_op* op, int k, int m, bool mixed);
sc_status related_solve(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m,
                        int freq, double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                        size_t work_bytes, hipStream_t s);

}  // namespace sc
