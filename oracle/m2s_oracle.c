/*
 * m2s_oracle.c -- CPU oracle for the matrix-free stencil solvers of
 * Mat2Stencil (sweeps with spatial loop-carried dependence, SpMV, multigrid
 * V-cycle and preconditioned CG).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded reference used to
 * check the HIP library.  It is built with -O2 -ffp-contract=off, shares no
 * code, header or constant with the library, and is loaded only by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg.
 *
 * Parity status of each part is recorded by the tests under tests/ that pin
 * it (assembled sparse matrices, triangular solves, closed forms, symmetry,
 * finite differences, exact elimination on a line for the VAR7 coarse
 * faces).  No routine is left unpinned.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define REAL double
#define SFX _f64
#include "m2s_oracle_impl.h"
#undef REAL
#undef SFX

#define REAL float
#define SFX _f32
#include "m2s_oracle_impl.h"
#undef REAL
#undef SFX

/* ------------------------------------------------------------------------
 * Preconditioned conjugate gradients in the form HPCG uses (Sec. 7.1; the
 * DSL's global scalars gathered with reduce_add, Sec. 4.4):
 *   r = b - A x
 *   repeat:  z = M^{-1} r
 *            rz = r.z ; p = z (first) or p = z + (rz / rz_old) p
 *            Ap = A p ; alpha = rz / (p.Ap)
 *            x += alpha p ; r -= alpha Ap
 *            stop when ||r|| / ||r0|| <= tol
 * When the recursive residual passes the test the true residual b - A x is
 * recomputed and replaces r; the loop only stops if that one passes too.
 * `replace_every` > 0 also replaces r by the true residual every that many
 * iterations.  All CG vectors and dot products are double; with
 * precond == 3 the V-cycle runs in float (r rounded to float on entry, z
 * widened to double on exit).
 * ---------------------------------------------------------------------- */
enum { PC_NONE = 0, PC_SYMGS = 1, PC_MG = 2, PC_MG_F32 = 3 };

typedef struct {
    int kind; /* 0 = CONST27, 1 = VAR7 */
    int nx, ny, nz;
    double diag, off;
    const double *kx, *ky, *kz;
} m2so_op;

static void op_apply(const m2so_op *A, const double *x, double *y)
{
    if (A->kind == 0)
        m2so_spmv27_f64(A->nx, A->ny, A->nz, A->diag, A->off, x, y);
    else
        m2so_spmv_var7_f64(A->nx, A->ny, A->nz, A->kx, A->ky, A->kz, x, y);
}

static double dot(long n, const double *a, const double *b)
{
    double s = 0;
    for (long p = 0; p < n; ++p) s += a[p] * b[p];
    return s;
}

/* Returns 0 converged (or max_iter reached with tol <= 0), 1 not converged,
 * 2 breakdown (p.Ap <= 0 or non-finite), -1 bad arguments.
 * hist (may be NULL) receives ||r_k|| / ||r_0|| for k = 0..iters. */
int m2so_pcg(int kind, int nx, int ny, int nz, double diag, double off,
             const double *kx, const double *ky, const double *kz,
             int precond, int mg_levels, const double *b, double *x,
             int max_iter, double tol, int replace_every, int *iters_out,
             double *relres_out, double *true_relres_out, double *hist)
{
    m2so_op A = {kind, nx, ny, nz, diag, off, kx, ky, kz};
    long n = (long)nx * ny * nz;
    m2so_mg__f64 *h64 = NULL;
    m2so_mg__f32 *h32 = NULL;
    float *kx32 = NULL, *ky32 = NULL, *kz32 = NULL, *r32 = NULL, *z32 = NULL;
    if (precond == PC_MG) {
        h64 = m2so_mg_create_f64(kind, mg_levels, nx, ny, nz, diag, off, kx,
                                 ky, kz);
        if (!h64) return -1;
    } else if (precond == PC_MG_F32) {
        if (kind == 1) {
            long fx = (long)nz * ny * (nx + 1), fy = (long)nz * (ny + 1) * nx,
                 fz = (long)(nz + 1) * ny * nx;
            kx32 = (float *)malloc(fx * sizeof(float));
            ky32 = (float *)malloc(fy * sizeof(float));
            kz32 = (float *)malloc(fz * sizeof(float));
            for (long t = 0; t < fx; ++t) kx32[t] = (float)kx[t];
            for (long t = 0; t < fy; ++t) ky32[t] = (float)ky[t];
            for (long t = 0; t < fz; ++t) kz32[t] = (float)kz[t];
        }
        h32 = m2so_mg_create_f32(kind, mg_levels, nx, ny, nz, (float)diag,
                                 (float)off, kx32, ky32, kz32);
        if (!h32) return -1;
        r32 = (float *)malloc(n * sizeof(float));
        z32 = (float *)malloc(n * sizeof(float));
    }
    double *r = (double *)malloc(n * sizeof(double));
    double *z = (double *)malloc(n * sizeof(double));
    double *p = (double *)malloc(n * sizeof(double));
    double *Ap = (double *)malloc(n * sizeof(double));

    op_apply(&A, x, Ap);
    for (long t = 0; t < n; ++t) r[t] = b[t] - Ap[t];
    double normr0 = sqrt(dot(n, r, r));
    double normr = normr0, rz = 0, rz_old = 0;
    int status = 1, it = 0;
    if (hist) hist[0] = 1.0;
    if (normr0 == 0) { status = 0; goto done; }

    for (it = 1; it <= max_iter; ++it) {
        if (precond == PC_NONE) {
            memcpy(z, r, n * sizeof(double));
        } else if (precond == PC_SYMGS) {
            memset(z, 0, n * sizeof(double));
            if (kind == 0) {
                m2so_symgs27_fwd_f64(nx, ny, nz, diag, off, r, z);
                m2so_symgs27_bwd_f64(nx, ny, nz, diag, off, r, z);
            } else {
                m2so_symgs_var7_fwd_f64(nx, ny, nz, kx, ky, kz, r, z);
                m2so_symgs_var7_bwd_f64(nx, ny, nz, kx, ky, kz, r, z);
            }
        } else if (precond == PC_MG) {
            m2so_mg_vcycle_f64(h64, r, z);
        } else {
            for (long t = 0; t < n; ++t) r32[t] = (float)r[t];
            m2so_mg_vcycle_f32(h32, r32, z32);
            for (long t = 0; t < n; ++t) z[t] = (double)z32[t];
        }
        rz_old = rz;
        rz = dot(n, r, z);
        if (it == 1) {
            memcpy(p, z, n * sizeof(double));
        } else {
            double beta = rz / rz_old;
            for (long t = 0; t < n; ++t) p[t] = z[t] + beta * p[t];
        }
        op_apply(&A, p, Ap);
        double pAp = dot(n, p, Ap);
        if (!(pAp > 0) || !isfinite(pAp)) { status = 2; break; }
        double alpha = rz / pAp;
        for (long t = 0; t < n; ++t) x[t] += alpha * p[t];
        for (long t = 0; t < n; ++t) r[t] -= alpha * Ap[t];
        normr = sqrt(dot(n, r, r));
        if (!isfinite(normr)) { status = 2; break; }
        int replace = replace_every > 0 && it % replace_every == 0;
        int check = tol > 0 && normr / normr0 <= tol;
        if (replace || check) {
            op_apply(&A, x, Ap);
            for (long t = 0; t < n; ++t) r[t] = b[t] - Ap[t];
            normr = sqrt(dot(n, r, r));
        }
        if (hist) hist[it] = normr / normr0;
        if (tol > 0 && normr / normr0 <= tol) { status = 0; break; }
    }
    if (it > max_iter) {
        it = max_iter;
        if (tol <= 0) status = 0;
    }
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = normr0 > 0 ? normr / normr0 : 0;
    if (true_relres_out) {
        op_apply(&A, x, Ap);
        for (long t = 0; t < n; ++t) r[t] = b[t] - Ap[t];
        *true_relres_out = normr0 > 0 ? sqrt(dot(n, r, r)) / normr0 : 0;
    }
    free(r);
    free(z);
    free(p);
    free(Ap);
    free(r32);
    free(z32);
    free(kx32);
    free(ky32);
    free(kz32);
    m2so_mg_destroy_f64(h64);
    m2so_mg_destroy_f32(h32);
    return status;
}
