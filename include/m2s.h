/*
 * m2s.h -- C ABI of the MI355X-native matrix-free stencil solver library
 * (libm2s.so): the hot path of Mat2Stencil's generated solvers, i.e. the
 * Seidel-style sweeps with spatial loop-carried dependence (lexicographic
 * Gauss-Seidel / SymGS and block SSOR), the Jacobi-style stencil SpMV beside
 * them, and the multigrid-preconditioned CG around both (paper Sec. 1,
 * Sec. 2.1.2, Sec. 4.3, Sec. 7.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.  A scalar field on an nx*ny*nz grid is a contiguous array stored
 *   [nz][ny][nx] (x fastest), point p = (k*ny + j)*nx + i; this is the
 *   paper's multi-dimensional row/column domain with the last index fastest
 *   (Sec. 4.2.1) and its "dictionary order" of domain loops (Sec. 4.4).
 *   "Lexicographic" = increasing p.  BLOCK7 fields carry 5 unknowns per
 *   point ("inner value as a tensor", Sec. 4.2.3), stored [nz][ny][nx][5].
 *   Values outside the grid are zero (Dirichlet), the padding matrix
 *   P = [0; I; 0] of Sec. 4.1 on every axis.
 * Memory.  Every vector / field / face-coefficient pointer is DEVICE memory
 *   owned by the caller, contiguous, of the stencil's dtype unless stated,
 *   and must stay valid until the stream work completes.  The library owns
 *   only the opaque m2s_workspace / m2s_mg objects (create/destroy).
 *   Host pointers are marked "host".
 * Streams.  All calls are asynchronous on the given hipStream_t (0 = the
 *   default stream) except m2s_pcg_solve, which synchronises and returns
 *   host-side results, and the create/destroy calls.
 * Errors.  Arguments are validated before anything is launched; a
 *   validation error returns a status and launches nothing.  A sweep's
 *   cross-workgroup wait is bounded: on expiry the kernel latches
 *   M2S_ERR_TIMEOUT in the workspace error word and exits; m2s_check()
 *   (synchronising) returns it.  No C++ exception crosses the ABI.
 * Threading.  Calls that share a workspace or MG object must be ordered on
 *   one stream.
 */
#ifndef M2S_H
#define M2S_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    M2S_OK = 0,
    M2S_ERR_ARG = 1,           /* null pointer, bad enum, bad option */
    M2S_ERR_SHAPE = 2,         /* extent <= 0, not coarsenable, too large */
    M2S_ERR_DTYPE = 3,         /* dtype not supported for this call */
    M2S_ERR_ALIAS = 4,         /* input and output vectors overlap */
    M2S_ERR_HIP = 5,           /* a HIP runtime call failed */
    M2S_ERR_TIMEOUT = 6,       /* a sweep's dependency wait expired */
    M2S_ERR_BREAKDOWN = 7,     /* CG: p.Ap <= 0 or a non-finite scalar */
    M2S_ERR_NOT_CONVERGED = 8, /* CG: max_iter reached above tolerance */
    M2S_ERR_UNSUPPORTED = 9    /* operator kind not valid for this call */
} m2s_status;

typedef enum { M2S_F64 = 0, M2S_F32 = 1 } m2s_dtype;

/* Operator kinds.
 * M2S_CONST27: HPCG-style 27-point operator (Sec. 7.1): `diag` on the
 *   diagonal, `offdiag` for each of the up to 26 in-grid neighbours.
 * M2S_VAR7: variable-coefficient diffusion D^T K D built from the
 *   difference and padding matrices of Sec. 4.1: (A u)_p = sum over the six
 *   faces f of p of k_f (u_p - u_q), u_q = 0 behind a boundary face.
 *   Face arrays (device, dtype): kx [nz][ny][nx+1] (face i between points
 *   i-1 and i), ky [nz][ny+1][nx], kz [nz+1][ny][nx].
 * M2S_BLOCK7_5: NPB-LU-shaped 7-point stencil with 5 unknowns per point and
 *   seven constant 5x5 blocks (host memory, 7*25 doubles, row-major, order
 *   centre, -x, +x, -y, +y, -z, +z): (A x)_p = B0 x_p + sum_d B_d x_{p+d}.
 *   F64 only. */
typedef enum { M2S_CONST27 = 0, M2S_VAR7 = 1, M2S_BLOCK7_5 = 2 } m2s_kind;

/* Sweep direction: forward = p ascending, backward = p descending,
 * symmetric = forward then backward (one SymGS / one SSOR iteration). */
typedef enum { M2S_FWD = 1, M2S_BWD = 2, M2S_SYM = 3 } m2s_dir;

typedef struct {
    int32_t nx, ny, nz;
} m2s_extent;

/* Matrix-free operator descriptor (the build's replacement for the paper's
 * row-function SpMat, Sec. 4.2: a fixed stencil over grid extents). */
typedef struct {
    m2s_kind kind;
    m2s_dtype dtype;      /* element type of vectors and face arrays */
    m2s_extent ext;
    double diag, offdiag; /* CONST27 only */
    const void *kx, *ky, *kz; /* VAR7 only: device face arrays */
    const double *blocks;     /* BLOCK7 only: HOST, 175 doubles */
} m2s_stencil;

typedef struct m2s_workspace m2s_workspace;
typedef struct m2s_mg m2s_mg;

/* Status text (static storage). */
const char *m2s_status_string(m2s_status s);

/* Library/ABI version, e.g. 10000 for 1.0.0. */
int m2s_version(void);

/* ---------------------------------------------------------------------
 * Workspace for the dependent sweeps: a ticket counter that hands tiles to
 * workgroups in dependency order; the tiles' boundary store, where each
 * boundary value is published once per launch as a record tagged with the
 * launch's epoch and polled by value by the dependent tiles (records are
 * never reset: a new epoch tells new records from old ones; the GPU
 * analogue of the monotone per-pair counters that Thm. 2 of Sec. 6.1 shows
 * are sufficient); a device error word; and scratch vectors of the
 * stencil's size (the out-of-place target of a half-sweep, adjoint
 * chains).  Allocates device memory at creation; a sweep whose plan needs
 * another tile layout (the tuning variables M2S_C27_WAVES / M2S_V7_WAVES
 * changed since) rebuilds the boundary store synchronously, and the first
 * m2s_symgs_xline call allocates that variant's record array.  One workspace serves one extent/kind/dtype;
 * calls using it must be stream-ordered.
 * --------------------------------------------------------------------- */
m2s_status m2s_workspace_create(const m2s_stencil *A, m2s_workspace **out);
void m2s_workspace_destroy(m2s_workspace *ws);

/* Synchronise `stream` and return the latched device error (M2S_OK,
 * M2S_ERR_TIMEOUT) or M2S_ERR_HIP; clears the latch. */
m2s_status m2s_check(m2s_workspace *ws, hipStream_t stream);

/* ---------------------------------------------------------------------
 * y = A x  (Sec. 4.3.1: sum over each row's non-zeros; Jacobi-style, no
 * spatial dependence).  Any kind; x and y must not overlap.
 * --------------------------------------------------------------------- */
m2s_status m2s_spmv(const m2s_stencil *A, const void *x, void *y,
                    hipStream_t stream);

/* y = L x (part = -1) or y = U x (part = +1): the strict lower / upper
 * triangle of A in lexicographic order.  CONST27 and VAR7.  Used by the
 * sweep adjoint. */
m2s_status m2s_spmv_part(const m2s_stencil *A, int part, const void *x,
                         void *y, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Gauss-Seidel sweeps in exact lexicographic order (Sec. 4.3.3, the
 * Seidel-style routine whose domain loop reads and writes the same vector;
 * SymGS = forward then backward, Sec. 1 and Sec. 7.1):
 *   x_p <- (r_p - sum_{q != p} a_pq x_q) / a_pp, p ascending (FWD) or
 *   descending (BWD), every neighbour taking its newest value.
 * CONST27 and VAR7, F64 and F32.  x is updated in place (via the
 * workspace's scratch vector); r is read-only; r and x must not overlap.
 * Executed as a persistent wavefront kernel: point (i, j, k) runs at step
 * i + 2j + 4k (CONST27) or i + j + k (VAR7) of the hyperplane schedule of
 * Sec. 6.1.3; tiles of 16 rows by 4 planes per wavefront are handed to
 * workgroups in dependency order and pass their boundary rows to their
 * neighbours as epoch-tagged records.  The result is bitwise identical to
 * the one-thread lexicographic sweep m2s_symgs_sequential (same per-point
 * arithmetic).
 * --------------------------------------------------------------------- */
m2s_status m2s_symgs(const m2s_stencil *A, const void *r, void *x,
                     m2s_dir dir, m2s_workspace *ws, hipStream_t stream);

/* Out-of-place half-sweep: x_out = sweep(r, x_in), dir FWD or BWD only.
 * x_in is not modified; x_in, x_out and r must not overlap. */
m2s_status m2s_symgs_oop(const m2s_stencil *A, const void *r,
                         const void *x_in, void *x_out, m2s_dir dir,
                         m2s_workspace *ws, hipStream_t stream);

/* Line-scheduled variant of the 27-point sweep (CONST27, F64 only; an
 * extension beyond the paper's schedules, built on the dependence
 * structure of the Seidel-style routine of Sec. 4.3.3 / Sec. 7.2.1).  Line
 * (j, k) is updated at step j + 2k of a line schedule; along the line the
 * recurrence x_i = g_i - (a_off / a_pp) x_{i-1} is solved by a parallel
 * prefix scan of affine maps.  Same update as m2s_symgs (in place, same
 * dir values, same workspace), but the scan regroups the sums: the result
 * equals the lexicographic sweep only up to rounding, not bitwise.  The
 * first call on a workspace allocates a 16-byte record per grid point in
 * it (the planes hand their new values to each other through them; freed
 * with the workspace).  Returns M2S_ERR_UNSUPPORTED for other kinds,
 * M2S_ERR_DTYPE for F32, M2S_ERR_SHAPE when nx > 4094 (the line does not
 * fit the scan's LDS) or nx*ny*nz >= 2^28, M2S_ERR_ALIAS if r and x
 * overlap, M2S_ERR_HIP if the record array cannot be allocated.  A
 * dependency wait that times out latches M2S_ERR_TIMEOUT (read by
 * m2s_check). */
m2s_status m2s_symgs_xline(const m2s_stencil *A, const void *r, void *x,
                           m2s_dir dir, m2s_workspace *ws, hipStream_t stream);

/* Reference: the same sweep run by ONE GPU thread in plain lexicographic
 * order, in place.  For testing the wavefront schedule only (slow). */
m2s_status m2s_symgs_sequential(const m2s_stencil *A, const void *r,
                                void *x, m2s_dir dir, hipStream_t stream);

/* Adjoint of one Gauss-Seidel half-sweep x_new = S(r, x_old) with respect
 * to its inputs, for a symmetric operator (CONST27, VAR7): given g = dL/dx_new
 *   FWD: gr = (D+L)^{-T} g = (D+U)^{-1} g  (a backward sweep from zero),
 *        gx = -U^T gr = -L gr
 *   BWD: gr = (D+L)^{-1} g (a forward sweep from zero), gx = -U gr
 * SYM (forward then backward) chains both in reverse order and returns the
 * summed gr and the gradient for the sweep's starting vector.  gr and gx
 * are outputs (overwritten); g is read-only; none may overlap.  The
 * transposed sweeps run on the same wavefront engine in reverse order. */
m2s_status m2s_symgs_adjoint(const m2s_stencil *A, const void *g, void *gr,
                             void *gx, m2s_dir dir, m2s_workspace *ws,
                             hipStream_t stream);

/* ---------------------------------------------------------------------
 * Block SSOR half-sweeps (the SSOR routine named in Sec. 1 and Sec. 4.3.3;
 * NPB-LU shape, Sec. 7.1) for BLOCK7_5, F64:
 *   x_p <- (1 - omega) x_p + omega B0^{-1} (b_p - sum_{d} B_d x_{p+d}),
 * p ascending (FWD) / descending (BWD) / FWD then BWD (SYM = one SSOR
 * iteration).  Per call the host factors B0 (LU with partial pivoting) and
 * forms omega B0^{-1} and omega B0^{-1} B_d, so a point is updated as
 *   x_p <- g_p - sum_{lower d} omega B0^{-1} B_d x_{p+d},
 *   g_p  = (1 - omega) x_p + omega B0^{-1} (b_p - sum_{upper d} B_d x_{p+d})
 * (lower / upper in sweep order), the same value up to rounding.  Executed
 * as a persistent wavefront kernel on the hyperplane i + j + k; x in place;
 * b read-only; b and x must not overlap.  Returns M2S_ERR_ARG if B0 is
 * singular or omega is not in (0, 2).
 * --------------------------------------------------------------------- */
m2s_status m2s_ssor_sweep(const m2s_stencil *A, const void *b, void *x,
                          double omega, m2s_dir dir, m2s_workspace *ws,
                          hipStream_t stream);

/* Reference: the same block SSOR sweep run by ONE GPU thread in plain
 * lexicographic order, in place, with the same per-point arithmetic.  For
 * testing the wavefront schedule only (slow); errors as m2s_ssor_sweep. */
m2s_status m2s_ssor_sweep_sequential(const m2s_stencil *A, const void *b,
                                     void *x, double omega, m2s_dir dir,
                                     hipStream_t stream);

/* ---------------------------------------------------------------------
 * Multigrid V-cycle (the HPCG MG of Sec. 7.1): levels obtained by halving
 * every extent (extents must be divisible by 2^(levels-1)); injection
 * restriction and prolongation (coarse point I on fine point 2I, the
 * "HPCG Prolong" matrix of Table 1); per level z = 0, one SymGS, fused
 * residual + restriction, recurse, prolongation, one SymGS; the coarsest
 * level runs one SymGS from zero.  CONST27 keeps the same stencil on every
 * level; a VAR7 coarse face gets half the conductance that exact
 * elimination of the fine points it spans gives on a 1-D line: ab/(2(a+b))
 * for two fine faces a, b in series (interior and last faces), k0/2 for the
 * first face, which spans fine face 0 alone.
 * prec = M2S_F32 runs the whole V-cycle in float (stored and computed):
 * m2s_mg_vcycle then takes r and returns z in DOUBLE and converts at the
 * boundary.  With prec = M2S_F64 r and z are double.
 * `fine` must be CONST27 or VAR7 with dtype F64; VAR7 face arrays are read
 * at create time only (copied/converted into library-owned storage).
 * --------------------------------------------------------------------- */
m2s_status m2s_mg_create(const m2s_stencil *fine, int levels, m2s_dtype prec,
                         m2s_mg **out);
m2s_status m2s_mg_vcycle(m2s_mg *mg, const double *r, double *z,
                         hipStream_t stream);
void m2s_mg_destroy(m2s_mg *mg);

/* ---------------------------------------------------------------------
 * Preconditioned CG in the HPCG form (Sec. 7.1; global scalars reduced as
 * the DSL's reduce_add, Sec. 4.4), all CG vectors and dot products double:
 *   r = b - A x; repeat { z = M^{-1} r; rz = r.z; p = z + (rz/rz_old) p
 *   (p = z first); Ap = A p; alpha = rz/(p.Ap); x += alpha p;
 *   r -= alpha Ap } until ||r||/||r0|| <= rtol.
 * When the recursive residual passes, r is replaced by the true residual
 * b - A x and the test repeated; replace_every > 0 also replaces it every
 * that many iterations.  rtol <= 0 runs exactly max_iter iterations.
 * Dot products are deterministic (fixed two-stage reduction order).
 * A: CONST27 or VAR7, F64.  precond: NONE, SYMGS (one SymGS from zero) or
 * MG (needs `mg` built on the same operator).  x holds x0 on entry and the
 * solution on return.  Synchronises `stream`.  Returns M2S_OK on
 * convergence (or after max_iter with rtol <= 0), M2S_ERR_NOT_CONVERGED,
 * M2S_ERR_BREAKDOWN, M2S_ERR_TIMEOUT.  The scalars are read back for the
 * convergence and breakdown tests every check_every iterations (values
 * <= 1 mean every iteration), at residual replacements and after the last
 * iteration; a run with a history reads them every iteration, and a
 * fixed-iteration run (rtol <= 0) without history or replacement only
 * after the last one.  Between read-backs the host does not wait, and a
 * breakdown (p.Ap <= 0 or a non-finite scalar) is latched on the device;
 * a converged solve reports the first checked iteration that passes (at
 * most check_every - 1 iterations past the first one that does).
 * Either way a breakdown leaves x at the last iterate before the failing
 * update (from that iteration on the update kernels leave x, r and p
 * alone) and iters is the iteration that broke down.
 * m2s_pcg_solve allocates its CG vectors (and, for SYMGS, a sweep
 * workspace) on every call and frees them before returning;
 * m2s_pcg_solve_ws takes them from a workspace made once with
 * m2s_pcg_workspace_create for an operator of the same kind and extent, and
 * allocates nothing (M2S_ERR_SHAPE for another kind or extent, M2S_ERR_ALIAS
 * if b or x is one of its vectors).  One workspace serves one solve at a
 * time; m2s_pcg_workspace_destroy synchronises the device first.
 * --------------------------------------------------------------------- */
typedef enum {
    M2S_PC_NONE = 0,
    M2S_PC_SYMGS = 1,
    M2S_PC_MG = 2
} m2s_precond;

typedef struct {
    int max_iter;
    double rtol;
    int replace_every;
    int check_every;   /* convergence read-back period; <= 1: every iteration */
} m2s_pcg_opts;

typedef struct {
    int iters;
    double rel_res;      /* ||r_k|| / ||r_0||, recursive (or replaced) */
    double true_rel_res; /* ||b - A x|| / ||r_0||, recomputed at the end */
    double r0_norm;
    int status;
    double seconds;      /* host wall time inside the call */
} m2s_pcg_info;

m2s_status m2s_pcg_solve(const m2s_stencil *A, m2s_precond precond,
                         m2s_mg *mg, const double *b, double *x,
                         const m2s_pcg_opts *opts, m2s_pcg_info *info,
                         double *hist /* host, max_iter+1 or NULL */,
                         hipStream_t stream);

typedef struct m2s_pcg_workspace m2s_pcg_workspace;
m2s_status m2s_pcg_workspace_create(const m2s_stencil *A,
                                    m2s_pcg_workspace **out);
void m2s_pcg_workspace_destroy(m2s_pcg_workspace *ws);
m2s_status m2s_pcg_solve_ws(const m2s_stencil *A, m2s_precond precond,
                            m2s_mg *mg, const double *b, double *x,
                            const m2s_pcg_opts *opts, m2s_pcg_info *info,
                            double *hist, m2s_pcg_workspace *ws,
                            hipStream_t stream);

/* ---------------------------------------------------------------------
 * Gradient with respect to the VAR7 face coefficients of a loss whose
 * derivative with respect to the solution u of A(k) u = f has adjoint
 * lam = A^{-T} dL/du:  dL/dk_f = -(lam_p - lam_q)(u_p - u_q), zero ghosts.
 * Outputs have the face-array shapes; F64.
 * --------------------------------------------------------------------- */
m2s_status m2s_face_grad(const m2s_stencil *A, const double *u,
                         const double *lam, double *gkx, double *gky,
                         double *gkz, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Small vector kernels used around the solvers (double, device):
 * m2s_dot writes x.y (fixed-order two-stage reduction) to *out (device);
 *   each call takes its own partials buffer from the stream-ordered
 *   allocator (hipMallocAsync / hipFreeAsync on `stream`), so concurrent
 *   calls do not share scratch.  n >= 0; M2S_ERR_HIP if that fails.
 * m2s_convert copies n elements between F64 and F32 (round to nearest).
 * --------------------------------------------------------------------- */
m2s_status m2s_dot(const double *x, const double *y, int64_t n, double *out,
                   hipStream_t stream);
m2s_status m2s_convert(const void *src, m2s_dtype src_t, void *dst,
                       m2s_dtype dst_t, int64_t n, hipStream_t stream);

/* ---------------------------------------------------------------------
 * m2s_dot_noalloc: m2s_dot for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and reduction order, so the
 * same bits as m2s_dot; it calls no allocator.  Its reduction scratch (1024
 * per-block partial sums and a counter: 1032 doubles, 8256 bytes) is a
 * fixed device array of the library, one per GPU, held from the first call
 * on that GPU until the process ends; the call clears the counter itself.
 * Any n >= 0 fits (the partials do not grow with n); should the reduction
 * ever need more partials than the array holds, the call returns
 * M2S_ERR_UNSUPPORTED.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (concurrent streams, threads) race and must be
 * ordered by the caller.  M2S_ERR_ARG for null pointers or n < 0.
 * --------------------------------------------------------------------- */
m2s_status m2s_dot_noalloc(const double *x, const double *y, int64_t n,
                           double *out, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Reference streaming passes for measurement (not a step of the method):
 * kind 0 copies c = a, kind 1 is the STREAM triad c = a + s*b, over n
 * doubles (device, 16-byte aligned; c must not overlap a or b).  They give
 * the HBM rate a plain streaming kernel reaches (bytes moved: 16 n for the
 * copy, 24 n for the triad), against which the sweeps' rates are also
 * reported.  M2S_ERR_ARG for another kind, a null or misaligned pointer or
 * n < 0; M2S_ERR_ALIAS for overlap.
 * --------------------------------------------------------------------- */
m2s_status m2s_stream(int32_t kind, const double *a, const double *b,
                      double *c, double s, int64_t n, hipStream_t stream);

/* ---------------------------------------------------------------------
 * ILU(0) of the 27-point operator (the incomplete LU of the ILU
 * microbenchmark, Sec. 7.2.1, as the paper cites it, Sec. 9), CONST27 F64:
 * L unit lower and U upper triangular with the sparsity pattern of A, by
 * row-wise (IKJ) Gaussian elimination in lexicographic order with every
 * fill-in outside the pattern dropped, so that (L U)_pq = a_pq on the
 * pattern.  Factor arrays per point p (C order of nz, ny, nx): L[13 p + a]
 * = l_pq for the 13 lower offsets, U[14 p] = u_pp and U[14 p + 1 + b] =
 * u_pq for the 13 upper offsets, offsets in lexicographic (dk, dj, di)
 * order, 0 outside the grid (caller-owned device arrays of 13 n and 14 n
 * doubles).  m2s_ilu0_apply computes z = (L U)^{-1} r: the lower solve
 * (p ascending), then the upper solve in place on z (p descending).  Both
 * run hyperplane by hyperplane (T = i + 2j + 4k, one launch per step), so
 * a call queues 7n - 6 (factor) or 2(7n - 6) (apply) launches for n^3.
 * M2S_ERR_UNSUPPORTED for other kinds, M2S_ERR_DTYPE for F32,
 * M2S_ERR_ALIAS if L and U overlap or z overlaps r, L or U.
 * --------------------------------------------------------------------- */
m2s_status m2s_ilu0_factor(const m2s_stencil *A, double *L, double *U,
                           hipStream_t stream);
m2s_status m2s_ilu0_apply(const m2s_stencil *A, const double *L,
                          const double *U, const double *r, double *z,
                          hipStream_t stream);

/* ---------------------------------------------------------------------
 * The same solves z = (L U)^{-1} r (Saad's ILU(0), Sec. 9) as persistent
 * band wavefronts, for ny <= 512: a workgroup owns a band of kt planes
 * (kt = min(nz, 512 / ny)), one lane per row, and walks it on the band's
 * hyperplanes i + 2j + 4kk with an LDS ring of each row's last 8 new values;
 * the band's top plane reaches the band above through epoch-tagged records
 * in the workspace.  The upper solve runs on the mirrored grid.
 * m2s_ilu0_pack copies the factor of m2s_ilu0_factor into the layout these
 * solves read (caller-owned Lp of 13 n and Up of 14 n doubles: per plane
 * and coefficient, the points of each diagonal i + 2j consecutive in j;
 * Up holds 1 / u_pp in place of u_pp), once per factor.
 * m2s_ilu0_apply_packed computes z from r with the packed factor: r is
 * copied into the packed order and the solves' results kept there (the
 * workspace's two scratch vectors: the upper solve's packed order is the
 * lower one's reversed), z written back in natural order.  Results
 * agree with m2s_ilu0_apply to rounding (ten of a point's 13 products are
 * summed a step early, the rest added in the step; not bitwise).
 * M2S_ERR_UNSUPPORTED for another kind or ny > 512, M2S_ERR_DTYPE for F32,
 * M2S_ERR_SHAPE past 32-bit byte offsets (14 n doubles, or the records), M2S_ERR_ALIAS
 * for overlapping arrays, M2S_ERR_TIMEOUT (via m2s_check) if a band waits
 * past the spin limit.  A workspace serves one solve at a time.
 * --------------------------------------------------------------------- */
m2s_status m2s_ilu0_pack(const m2s_stencil *A, const double *L,
                         const double *U, double *Lp, double *Up,
                         m2s_workspace *ws, hipStream_t stream);
m2s_status m2s_ilu0_apply_packed(const m2s_stencil *A, const double *Lp,
                                 const double *Up, const double *r, double *z,
                                 m2s_workspace *ws, hipStream_t stream);

/* ---------------------------------------------------------------------
 * D-ILU of the 27-point operator (the factored-diagonal incomplete
 * factorisation: A's off-diagonals kept, only the diagonal factored; not
 * ILU(0), see above), CONST27 F64: M = (D + L) D^{-1} (D + U) with L, U the
 * strict lower and
 * upper parts of A and the diagonal D = diag(d) factored so that
 * diag(M) = diag(A):  d_p = diag - sum_{q lower} off^2 / d_q.
 * m2s_dilu27_factor writes w = 1/d (n doubles, caller-owned).
 * m2s_dilu27_apply computes z = M^{-1} r: the lower solve
 *   y_p = (r_p - off sum_{q lower} y_q) / d_p,  p ascending,
 * into the workspace's scratch vector, then the upper solve
 *   z_p = y_p - off (sum_{q upper} z_q) / d_p,  p descending.
 * All three are exact lexicographic sweeps over the 13 lower neighbours in
 * sweep order, run on the 27-point wavefront tiles (1 or 2 compute
 * wavefronts per tile, M2S_ERR_HIP otherwise).  r, w, z must not overlap.
 * --------------------------------------------------------------------- */
m2s_status m2s_dilu27_factor(const m2s_stencil *A, void *w, m2s_workspace *ws,
                            hipStream_t stream);
m2s_status m2s_dilu27_apply(const m2s_stencil *A, const void *w,
                           const void *r, void *z, m2s_workspace *ws,
                           hipStream_t stream);

/* ---------------------------------------------------------------------
 * Jacobi iterations of the 2-D 9-point operator (the JacIter
 * microbenchmark of Sec. 7.2.1): on an nx x ny grid ([ny][nx], x fastest,
 * F64), iters times
 *   x_p <- (b_p - off * sum_{q in N8(p)} x_q) / diag,
 * all points at once from the previous iterate; values outside the grid
 * are 0 (Dirichlet).  x: in x_0, out x_iters; b read-only; tmp: a second
 * nx*ny-double device buffer owned by the caller (overwritten).  tblock
 * (1, 2, 4 or 8): iterations fused per pass over memory (temporal blocking
 * in LDS; the result does not depend on it beyond rounding order).  x, b
 * and tmp must not overlap; nx*ny < 2^31; diag != 0.
 * --------------------------------------------------------------------- */
m2s_status m2s_jacobi9(int32_t nx, int32_t ny, double diag, double off,
                       const double *b, double *x, double *tmp, int32_t iters,
                       int32_t tblock, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Pentadiagonal line solves (the scalar multi-diagonal systems of the
 * ADI-shaped NPB SP solver, Sec. 7.1): along axis 0 (x), 1 (y) or 2 (z)
 * every grid line of an nx x ny x nz grid ([nz][ny][nx], F64) holds
 *   a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2} = r_i
 * (i the position on the line; terms reaching off the line are ignored).
 * coef: 5 consecutive fields a, b, c, d, e (5 n doubles); r: n doubles;
 * x: the solution (n doubles, overwritten); work: 2 n doubles of caller-
 * owned scratch (overwritten).  Gaussian elimination without pivoting
 * (the systems must be safe for it, e.g. diagonally dominant), one line per
 * GPU lane (chunks of each line staged through LDS), elimination and back
 * substitution in one launch.  None of the four buffers may overlap;
 * n < 2^31.
 * --------------------------------------------------------------------- */
m2s_status m2s_penta_lines(int32_t nx, int32_t ny, int32_t nz, int32_t axis,
                           const double *coef, const double *r, double *x,
                           double *work, hipStream_t stream);

/* ---------------------------------------------------------------------
 * 5x5 block-tridiagonal line solves (the block systems of the ADI-shaped
 * NPB BT solver, Sec. 7.1): along axis 0 (x), 1 (y) or 2 (z) every grid
 * line of an nx x ny x nz grid holds
 *   A_i x_{i-1} + B_i x_i + C_i x_{i+1} = r_i
 * in 5-vectors x_i, r_i with 5x5 blocks (i the position on the line; the
 * first point's A and the last point's C couple to nothing and are not
 * read).  coef: device, F64, [3][nz][ny][nx][5][5] = A, B, C at every
 * point, blocks row-major (75 n doubles); r: [nz][ny][nx][5] (5 n
 * doubles); x: the solution, same layout (overwritten); work: 25 n doubles
 * of caller-owned scratch (overwritten).  Block Gaussian elimination down
 * each line (G_i = M_i^{-1} C_i, y_i = M_i^{-1}(r_i - A_i y_{i-1}),
 * M_i = B_i - A_i G_{i-1}) and back substitution x_i = y_i - G_i x_{i+1},
 * one line per GPU lane, both passes in one launch.  The pivot blocks M_i
 * are factored without pivoting: the systems must keep them safely
 * nonsingular (e.g. block diagonal dominance); a zero pivot gives
 * non-finite values, not an error.  None of the four buffers may overlap
 * (M2S_ERR_ALIAS); n = nx*ny*nz < 2^31 (M2S_ERR_SHAPE); null pointers or an
 * axis outside 0..2 give M2S_ERR_ARG.
 * --------------------------------------------------------------------- */
m2s_status m2s_bt_lines(int32_t nx, int32_t ny, int32_t nz, int32_t axis,
                        const double *coef, const double *r, double *x,
                        double *work, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Schedule of the wavefront sweep (host only, no GPU needed), exposed so
 * the schedule's legality (every dependence from a strictly earlier step)
 * can be checked on the CPU.  Point (i, j, k) runs at step
 * i + lag_row*j + lag_plane*k (the hyperplane of Sec. 6.1.3).
 * M2S_CONST27: the grid's rows (j, k) are cut into tiles of row_slots = 16
 *   consecutive u = j + k by slab_planes consecutive k (4 per wavefront),
 *   one lane per row; nslabs = number of tiles holding a grid row, taken in
 *   lexicographic (k-tile, u-tile) order; steps = steps of a full tile.
 * M2S_VAR7, M2S_BLOCK7_5: tiles of row_slots = 16 consecutive j by
 *   slab_planes consecutive k, one lane per row; nslabs = number of tiles,
 *   taken in lexicographic (k-tile, j-tile) order; steps = steps of a full
 *   tile.
 * threads = workgroup size; publish_every = 1 (tiles hand over their
 * boundary rows every step).
 * --------------------------------------------------------------------- */
typedef struct {
    int32_t slab_planes, nslabs, row_slots, lag_row, lag_plane, steps;
    int32_t threads, publish_every;
} m2s_sweep_plan;

m2s_status m2s_plan_sweep(const m2s_stencil *A, m2s_sweep_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* M2S_H */
