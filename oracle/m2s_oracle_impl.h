/*
 * m2s_oracle_impl.h -- body of the CPU oracle, instantiated once per
 * floating-point type by m2s_oracle.c (REAL = double, then REAL = float).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library never does.  It shares no code with the library.
 *
 * Grid convention (the paper's multi-dimensional domains with the last index
 * fastest, Sec. 4.2.1 "Multi-dimensional rows and columns"; domain loops run
 * in dictionary order, Sec. 4.4 grammar): a scalar field on an nx*ny*nz grid
 * is stored as [nz][ny][nx], p = (k*ny + j)*nx + i, and "lexicographic"
 * means increasing p.  Values outside the grid are zero (Dirichlet), which is
 * the padding matrix P = [0; I; 0] of Sec. 4.1 applied to every axis.
 *
 * Every function is written as the plain definition of what it computes.
 * Summation orders are fixed and documented; no blocking, fusion or
 * reordering beyond the definition.
 */

#ifndef REAL
#error "define REAL and SFX before including this file"
#endif

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(m2so_, CAT(name, SFX))

static inline long CAT(idx3_, SFX)(int nx, int ny, int i, int j, int k)
{
    return ((long)k * ny + j) * nx + i;
}
#define IDX(i, j, k) CAT(idx3_, SFX)(nx, ny, (i), (j), (k))

/* ------------------------------------------------------------------------
 * CONST27: the HPCG-style 27-point operator.  Row p has `diag` on the
 * diagonal and `off` for each of the (up to) 26 in-grid neighbours
 * q in N27(p).  Sec. 7.1 (HPCG end-to-end case), Sec. 4.3.1 (SpMV is the
 * sum over the row's non-zeros of value times vector entry).
 * Summation order: diagonal first, then neighbours in lexicographic offset
 * order (dz, dy, dx each from -1 to +1).
 * ---------------------------------------------------------------------- */
void FN(spmv27)(int nx, int ny, int nz, REAL diag, REAL off,
                const REAL *x, REAL *y)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL s = diag * x[IDX(i, j, k)];
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int ii = i + dx, jj = j + dy, kk = k + dz;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny ||
                                kk < 0 || kk >= nz)
                                continue;
                            s += off * x[IDX(ii, jj, kk)];
                        }
                y[IDX(i, j, k)] = s;
            }
}

/* One Gauss-Seidel update of point (i,j,k) in place:
 *   x_p <- (r_p - sum_{q != p} a_pq x_q) / a_pp
 * reading whatever x currently holds (new values for points already visited
 * in this sweep, old values for the rest).  Sec. 4.3.3 (routines whose domain
 * loop reads and writes the same vector), textbook Gauss-Seidel. */
static void CAT(gs27_point_, SFX)(int nx, int ny, int nz, REAL diag, REAL off,
                                  const REAL *r, REAL *x, int i, int j, int k)
{
    REAL s = r[IDX(i, j, k)];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                    kk >= nz)
                    continue;
                s -= off * x[IDX(ii, jj, kk)];
            }
    x[IDX(i, j, k)] = s / diag;
}

/* Forward lexicographic sweep: p ascending. */
void FN(symgs27_fwd)(int nx, int ny, int nz, REAL diag, REAL off,
                     const REAL *r, REAL *x)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                CAT(gs27_point_, SFX)(nx, ny, nz, diag, off, r, x, i, j, k);
}

/* Backward lexicographic sweep: p descending. */
void FN(symgs27_bwd)(int nx, int ny, int nz, REAL diag, REAL off,
                     const REAL *r, REAL *x)
{
    for (int k = nz - 1; k >= 0; --k)
        for (int j = ny - 1; j >= 0; --j)
            for (int i = nx - 1; i >= 0; --i)
                CAT(gs27_point_, SFX)(nx, ny, nz, diag, off, r, x, i, j, k);
}

/* Strict lower (part = -1) or strict upper (part = +1) triangle of the
 * CONST27 operator applied to x: y_p = sum over neighbours q of p with
 * q < p (resp. q > p) in lexicographic order of off * x_q.  Used for the
 * adjoint of a sweep with respect to its starting vector. */
void FN(spmv27_part)(int nx, int ny, int nz, REAL off, int part,
                     const REAL *x, REAL *y)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL s = 0;
                long p = IDX(i, j, k);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int ii = i + dx, jj = j + dy, kk = k + dz;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny ||
                                kk < 0 || kk >= nz)
                                continue;
                            long q = IDX(ii, jj, kk);
                            if ((part < 0 && q < p) || (part > 0 && q > p))
                                s += off * x[q];
                        }
                y[p] = s;
            }
}

/* ------------------------------------------------------------------------
 * VAR7: variable-coefficient 7-point diffusion, the operator D^T K D built
 * from the difference matrix D and padding P of Sec. 4.1 on each axis, with
 * one coefficient per cell face:
 *   (A u)_p = sum over the 6 faces f of p of k_f (u_p - u_q),
 * where u_q = 0 for the ghost point behind a boundary face.
 * Face arrays: kx[nz][ny][nx+1] (face i sits between points i-1 and i),
 *              ky[nz][ny+1][nx], kz[nz+1][ny][nx].
 * Term order: centre (sum of the six faces times u_p) then -x, +x, -y, +y,
 * -z, +z neighbours.
 * ---------------------------------------------------------------------- */
#define KX(i, j, k) kx[((long)(k) * ny + (j)) * (nx + 1) + (i)]
#define KY(i, j, k) ky[((long)(k) * (ny + 1) + (j)) * nx + (i)]
#define KZ(i, j, k) kz[((long)(k) * ny + (j)) * nx + (i)]

static inline REAL CAT(var7_diag_, SFX)(int nx, int ny, const REAL *kx,
                                        const REAL *ky, const REAL *kz, int i,
                                        int j, int k)
{
    return KX(i, j, k) + KX(i + 1, j, k) + KY(i, j, k) + KY(i, j + 1, k) +
           KZ(i, j, k) + KZ(i, j, k + 1);
}

/* Off-diagonal entries of row p, in the fixed order -x,+x,-y,+y,-z,+z.
 * Writes the neighbour flat index (or -1 if outside) and a_pq = -k_f. */
static inline void CAT(var7_row_, SFX)(int nx, int ny, int nz, const REAL *kx,
                                       const REAL *ky, const REAL *kz, int i,
                                       int j, int k, long q[6], REAL a[6])
{
    q[0] = i > 0 ? IDX(i - 1, j, k) : -1;      a[0] = -KX(i, j, k);
    q[1] = i < nx - 1 ? IDX(i + 1, j, k) : -1; a[1] = -KX(i + 1, j, k);
    q[2] = j > 0 ? IDX(i, j - 1, k) : -1;      a[2] = -KY(i, j, k);
    q[3] = j < ny - 1 ? IDX(i, j + 1, k) : -1; a[3] = -KY(i, j + 1, k);
    q[4] = k > 0 ? IDX(i, j, k - 1) : -1;      a[4] = -KZ(i, j, k);
    q[5] = k < nz - 1 ? IDX(i, j, k + 1) : -1; a[5] = -KZ(i, j, k + 1);
}

void FN(spmv_var7)(int nx, int ny, int nz, const REAL *kx, const REAL *ky,
                   const REAL *kz, const REAL *x, REAL *y)
{
    long q[6];
    REAL a[6];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL s = CAT(var7_diag_, SFX)(nx, ny, kx, ky, kz, i, j, k) *
                         x[IDX(i, j, k)];
                CAT(var7_row_, SFX)(nx, ny, nz, kx, ky, kz, i, j, k, q, a);
                for (int d = 0; d < 6; ++d)
                    if (q[d] >= 0) s += a[d] * x[q[d]];
                y[IDX(i, j, k)] = s;
            }
}

/* Strict lower (part = -1) or upper (part = +1) triangle of VAR7 times x. */
void FN(spmv_var7_part)(int nx, int ny, int nz, const REAL *kx,
                        const REAL *ky, const REAL *kz, int part,
                        const REAL *x, REAL *y)
{
    long q[6];
    REAL a[6];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = IDX(i, j, k);
                REAL s = 0;
                CAT(var7_row_, SFX)(nx, ny, nz, kx, ky, kz, i, j, k, q, a);
                for (int d = 0; d < 6; ++d)
                    if (q[d] >= 0 && ((part < 0 && q[d] < p) ||
                                      (part > 0 && q[d] > p)))
                        s += a[d] * x[q[d]];
                y[p] = s;
            }
}

static void CAT(gs7_point_, SFX)(int nx, int ny, int nz, const REAL *kx,
                                 const REAL *ky, const REAL *kz,
                                 const REAL *r, REAL *x, int i, int j, int k)
{
    long q[6];
    REAL a[6];
    CAT(var7_row_, SFX)(nx, ny, nz, kx, ky, kz, i, j, k, q, a);
    REAL s = r[IDX(i, j, k)];
    for (int d = 0; d < 6; ++d)
        if (q[d] >= 0) s -= a[d] * x[q[d]];
    x[IDX(i, j, k)] = s / CAT(var7_diag_, SFX)(nx, ny, kx, ky, kz, i, j, k);
}

void FN(symgs_var7_fwd)(int nx, int ny, int nz, const REAL *kx,
                        const REAL *ky, const REAL *kz, const REAL *r,
                        REAL *x)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                CAT(gs7_point_, SFX)(nx, ny, nz, kx, ky, kz, r, x, i, j, k);
}

void FN(symgs_var7_bwd)(int nx, int ny, int nz, const REAL *kx,
                        const REAL *ky, const REAL *kz, const REAL *r,
                        REAL *x)
{
    for (int k = nz - 1; k >= 0; --k)
        for (int j = ny - 1; j >= 0; --j)
            for (int i = nx - 1; i >= 0; --i)
                CAT(gs7_point_, SFX)(nx, ny, nz, kx, ky, kz, r, x, i, j, k);
}

/* Coarse VAR7 coefficients for a grid coarsened by 2 per axis with
 * injection (coarse point I sits on fine point 2I).  The paper fixes no rule
 * for this; the reading used here: each coarse face gets 1/2 of the
 * conductance that exact elimination of the fine points between the two
 * coarse points (or between the coarse point and the Dirichlet ghost) gives
 * on a 1-D line, i.e. of the Schur complement of D^T K D (Sec. 4.1) onto the
 * even points.  Two fine faces a, b in series give ab/(a+b), so an interior
 * coarse face I (fine faces 2I-1 and 2I) and the last one (fine faces nf-1
 * and nf) get ab/(2(a+b)), a quarter of their harmonic mean.  The first
 * coarse face has no fine point to eliminate: fine point 0 is coarse point
 * 0 and touches the ghost through fine face 0 alone, so it gets k0/2.  The
 * factor 1/2 is one constant on every face: it is 1/4 for the injected
 * residual (the operator carries no 1/h^2) times 2 for the coarse face being
 * twice the fine face in area per unit length.  Transverse position: the
 * fine face row through the coincident fine points (2J, 2K). */
static inline REAL CAT(half_series_, SFX)(REAL a, REAL b)
{
    return (a * b) / ((REAL)2 * (a + b));
}

void FN(var7_coarsen)(int nx, int ny, int nz, const REAL *kx, const REAL *ky,
                      const REAL *kz, REAL *kxc, REAL *kyc, REAL *kzc)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I <= cx; ++I) {
                REAL v;
                if (I == 0) v = KX(0, 2 * J, 2 * K) / (REAL)2;
                else v = CAT(half_series_, SFX)(KX(2 * I - 1, 2 * J, 2 * K),
                                                KX(2 * I, 2 * J, 2 * K));
                kxc[((long)K * cy + J) * (cx + 1) + I] = v;
            }
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J <= cy; ++J)
            for (int I = 0; I < cx; ++I) {
                REAL v;
                if (J == 0) v = KY(2 * I, 0, 2 * K) / (REAL)2;
                else v = CAT(half_series_, SFX)(KY(2 * I, 2 * J - 1, 2 * K),
                                                KY(2 * I, 2 * J, 2 * K));
                kyc[((long)K * (cy + 1) + J) * cx + I] = v;
            }
    for (int K = 0; K <= cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                REAL v;
                if (K == 0) v = KZ(2 * I, 2 * J, 0) / (REAL)2;
                else v = CAT(half_series_, SFX)(KZ(2 * I, 2 * J, 2 * K - 1),
                                                KZ(2 * I, 2 * J, 2 * K));
                kzc[((long)K * cy + J) * cx + I] = v;
            }
}

/* Gradient of L with respect to the face coefficients, given the solution u
 * of A(k) u = f and the adjoint lambda = A^{-T} dL/du:
 *   dL/dk_f = -lambda^T (dA/dk_f) u = -(lambda_p - lambda_q)(u_p - u_q)
 * with lambda_q = u_q = 0 behind a boundary face. */
void FN(var7_face_grad)(int nx, int ny, int nz, const REAL *u,
                        const REAL *lam, REAL *gx, REAL *gy, REAL *gz)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                REAL ua = i > 0 ? u[IDX(i - 1, j, k)] : 0;
                REAL la = i > 0 ? lam[IDX(i - 1, j, k)] : 0;
                REAL ub = i < nx ? u[IDX(i, j, k)] : 0;
                REAL lb = i < nx ? lam[IDX(i, j, k)] : 0;
                gx[((long)k * ny + j) * (nx + 1) + i] = -(lb - la) * (ub - ua);
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL ua = j > 0 ? u[IDX(i, j - 1, k)] : 0;
                REAL la = j > 0 ? lam[IDX(i, j - 1, k)] : 0;
                REAL ub = j < ny ? u[IDX(i, j, k)] : 0;
                REAL lb = j < ny ? lam[IDX(i, j, k)] : 0;
                gy[((long)k * (ny + 1) + j) * nx + i] = -(lb - la) * (ub - ua);
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL ua = k > 0 ? u[IDX(i, j, k - 1)] : 0;
                REAL la = k > 0 ? lam[IDX(i, j, k - 1)] : 0;
                REAL ub = k < nz ? u[IDX(i, j, k)] : 0;
                REAL lb = k < nz ? lam[IDX(i, j, k)] : 0;
                gz[((long)k * ny + j) * nx + i] = -(lb - la) * (ub - ua);
            }
}

/* ------------------------------------------------------------------------
 * BLOCK7x5: five unknowns per point ("inner value as a tensor", Sec. 4.2.3),
 * stored [nz][ny][nx][5].  Seven constant 5x5 blocks, row-major, in the
 * order centre, -x, +x, -y, +y, -z, +z:
 *   (A x)_p = B0 x_p + sum_{d=1..6, p+d in grid} B_d x_{p+d}.
 * ---------------------------------------------------------------------- */
static const int CAT(b7_off_, SFX)[7][3] = {
    {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
    {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

void FN(spmv_block7)(int nx, int ny, int nz, const REAL *blk, const REAL *x,
                     REAL *y)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL s[5] = {0, 0, 0, 0, 0};
                for (int d = 0; d < 7; ++d) {
                    int ii = i + CAT(b7_off_, SFX)[d][0];
                    int jj = j + CAT(b7_off_, SFX)[d][1];
                    int kk = k + CAT(b7_off_, SFX)[d][2];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                        kk >= nz)
                        continue;
                    const REAL *xq = x + 5 * IDX(ii, jj, kk);
                    const REAL *B = blk + 25 * d;
                    for (int a = 0; a < 5; ++a)
                        for (int c = 0; c < 5; ++c) s[a] += B[5 * a + c] * xq[c];
                }
                for (int a = 0; a < 5; ++a) y[5 * IDX(i, j, k) + a] = s[a];
            }
}

/* LU factorisation with partial pivoting of a 5x5 block (Doolittle, row
 * interchanges recorded in piv).  lu holds L (unit, below the diagonal) and
 * U (on and above).  Returns 0, or -1 for an exactly singular pivot. */
int FN(lu5_factor)(const REAL *A, REAL *lu, int *piv)
{
    for (int t = 0; t < 25; ++t) lu[t] = A[t];
    for (int c = 0; c < 5; ++c) {
        int p = c;
        REAL best = lu[5 * c + c] < 0 ? -lu[5 * c + c] : lu[5 * c + c];
        for (int r = c + 1; r < 5; ++r) {
            REAL v = lu[5 * r + c] < 0 ? -lu[5 * r + c] : lu[5 * r + c];
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (best == 0) return -1;
        if (p != c)
            for (int t = 0; t < 5; ++t) {
                REAL tmp = lu[5 * c + t];
                lu[5 * c + t] = lu[5 * p + t];
                lu[5 * p + t] = tmp;
            }
        for (int r = c + 1; r < 5; ++r) {
            lu[5 * r + c] /= lu[5 * c + c];
            for (int t = c + 1; t < 5; ++t)
                lu[5 * r + t] -= lu[5 * r + c] * lu[5 * c + t];
        }
    }
    return 0;
}

/* Solve (P^T L U) y = s in place on y (y holds s on entry). */
void FN(lu5_solve)(const REAL *lu, const int *piv, REAL *y)
{
    for (int c = 0; c < 5; ++c)
        if (piv[c] != c) {
            REAL tmp = y[c];
            y[c] = y[piv[c]];
            y[piv[c]] = tmp;
        }
    for (int r = 1; r < 5; ++r)
        for (int c = 0; c < r; ++c) y[r] -= lu[5 * r + c] * y[c];
    for (int r = 4; r >= 0; --r) {
        for (int c = r + 1; c < 5; ++c) y[r] -= lu[5 * r + c] * y[c];
        y[r] /= lu[5 * r + r];
    }
}

/* One block SSOR relaxation of point (i,j,k) in place:
 *   x_p <- (1 - w) x_p + w B0^{-1} (b_p - sum_{d=1..6} B_d x_{p+d}). */
static void CAT(ssor_point_, SFX)(int nx, int ny, int nz, const REAL *blk,
                                  const REAL *lu, const int *piv, REAL w,
                                  const REAL *b, REAL *x, int i, int j, int k)
{
    REAL s[5];
    for (int a = 0; a < 5; ++a) s[a] = b[5 * IDX(i, j, k) + a];
    for (int d = 1; d < 7; ++d) {
        int ii = i + CAT(b7_off_, SFX)[d][0];
        int jj = j + CAT(b7_off_, SFX)[d][1];
        int kk = k + CAT(b7_off_, SFX)[d][2];
        if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz)
            continue;
        const REAL *xq = x + 5 * IDX(ii, jj, kk);
        const REAL *B = blk + 25 * d;
        for (int a = 0; a < 5; ++a)
            for (int c = 0; c < 5; ++c) s[a] -= B[5 * a + c] * xq[c];
    }
    FN(lu5_solve)(lu, piv, s);
    REAL *xp = x + 5 * IDX(i, j, k);
    for (int a = 0; a < 5; ++a) xp[a] = ((REAL)1 - w) * xp[a] + w * s[a];
}

int FN(ssor_block7_fwd)(int nx, int ny, int nz, const REAL *blk, REAL w,
                        const REAL *b, REAL *x)
{
    REAL lu[25];
    int piv[5];
    if (FN(lu5_factor)(blk, lu, piv)) return -1;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                CAT(ssor_point_, SFX)(nx, ny, nz, blk, lu, piv, w, b, x, i, j,
                                      k);
    return 0;
}

int FN(ssor_block7_bwd)(int nx, int ny, int nz, const REAL *blk, REAL w,
                        const REAL *b, REAL *x)
{
    REAL lu[25];
    int piv[5];
    if (FN(lu5_factor)(blk, lu, piv)) return -1;
    for (int k = nz - 1; k >= 0; --k)
        for (int j = ny - 1; j >= 0; --j)
            for (int i = nx - 1; i >= 0; --i)
                CAT(ssor_point_, SFX)(nx, ny, nz, blk, lu, piv, w, b, x, i, j,
                                      k);
    return 0;
}

/* ------------------------------------------------------------------------
 * Multigrid (Sec. 7.1, the HPCG solver): injection restriction and
 * prolongation between a fine grid and the grid coarsened by 2 per axis
 * (coarse point (I,J,K) coincides with fine point (2I,2J,2K); the "HPCG
 * Prolong" matrix of Table 1).
 * ---------------------------------------------------------------------- */

/* rc = (r - A z) sampled at the coincident fine points, A given as a matvec
 * already applied: az = A z on the fine grid. */
void FN(restrict_inject)(int nx, int ny, int nz, const REAL *r,
                         const REAL *az, REAL *rc)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                long f = IDX(2 * I, 2 * J, 2 * K);
                rc[((long)K * cy + J) * cx + I] = r[f] - az[f];
            }
}

/* z[2I,2J,2K] += zc[I,J,K]. */
void FN(prolong_inject)(int nx, int ny, int nz, const REAL *zc, REAL *z)
{
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I)
                z[IDX(2 * I, 2 * J, 2 * K)] += zc[((long)K * cy + J) * cx + I];
}

/* A multigrid hierarchy of one operator kind.  Level 0 is the finest. */
typedef struct {
    int kind; /* 0 = CONST27, 1 = VAR7 */
    int nlev;
    int nx[8], ny[8], nz[8];
    REAL diag, off;               /* CONST27: same stencil on every level */
    REAL *kx[8], *ky[8], *kz[8];  /* VAR7: owned face arrays per level */
    REAL *az[8], *rc[8], *zc[8];  /* work vectors: A z, coarse r, coarse z */
} CAT(m2so_mg_, SFX);

static void CAT(mg_apply_, SFX)(CAT(m2so_mg_, SFX) * h, int l, const REAL *x,
                                REAL *y)
{
    if (h->kind == 0)
        FN(spmv27)(h->nx[l], h->ny[l], h->nz[l], h->diag, h->off, x, y);
    else
        FN(spmv_var7)(h->nx[l], h->ny[l], h->nz[l], h->kx[l], h->ky[l],
                      h->kz[l], x, y);
}

static void CAT(mg_symgs_, SFX)(CAT(m2so_mg_, SFX) * h, int l, const REAL *r,
                                REAL *z)
{
    if (h->kind == 0) {
        FN(symgs27_fwd)(h->nx[l], h->ny[l], h->nz[l], h->diag, h->off, r, z);
        FN(symgs27_bwd)(h->nx[l], h->ny[l], h->nz[l], h->diag, h->off, r, z);
    } else {
        FN(symgs_var7_fwd)(h->nx[l], h->ny[l], h->nz[l], h->kx[l], h->ky[l],
                           h->kz[l], r, z);
        FN(symgs_var7_bwd)(h->nx[l], h->ny[l], h->nz[l], h->kx[l], h->ky[l],
                           h->kz[l], r, z);
    }
}

/* Build the hierarchy.  Returns NULL if an extent is not divisible by
 * 2^(nlev-1) or nlev is out of range.  For VAR7 the fine face arrays are
 * copied, the coarse ones derived by var7_coarsen. */
CAT(m2so_mg_, SFX) * FN(mg_create)(int kind, int nlev, int nx, int ny, int nz,
                                   REAL diag, REAL off, const REAL *kx,
                                   const REAL *ky, const REAL *kz)
{
    if (nlev < 1 || nlev > 8) return NULL;
    int f = 1 << (nlev - 1);
    if (nx % f || ny % f || nz % f) return NULL;
    CAT(m2so_mg_, SFX) *h = (CAT(m2so_mg_, SFX) *)calloc(1, sizeof(*h));
    h->kind = kind;
    h->nlev = nlev;
    h->diag = diag;
    h->off = off;
    for (int l = 0; l < nlev; ++l) {
        h->nx[l] = nx >> l;
        h->ny[l] = ny >> l;
        h->nz[l] = nz >> l;
        long n = (long)h->nx[l] * h->ny[l] * h->nz[l];
        h->az[l] = (REAL *)calloc(n, sizeof(REAL));
        if (l > 0) {
            h->rc[l] = (REAL *)calloc(n, sizeof(REAL));
            h->zc[l] = (REAL *)calloc(n, sizeof(REAL));
        }
        if (kind == 1) {
            long fx = (long)h->nz[l] * h->ny[l] * (h->nx[l] + 1);
            long fy = (long)h->nz[l] * (h->ny[l] + 1) * h->nx[l];
            long fz = (long)(h->nz[l] + 1) * h->ny[l] * h->nx[l];
            h->kx[l] = (REAL *)malloc(fx * sizeof(REAL));
            h->ky[l] = (REAL *)malloc(fy * sizeof(REAL));
            h->kz[l] = (REAL *)malloc(fz * sizeof(REAL));
            if (l == 0) {
                memcpy(h->kx[0], kx, fx * sizeof(REAL));
                memcpy(h->ky[0], ky, fy * sizeof(REAL));
                memcpy(h->kz[0], kz, fz * sizeof(REAL));
            } else {
                FN(var7_coarsen)(h->nx[l - 1], h->ny[l - 1], h->nz[l - 1],
                                 h->kx[l - 1], h->ky[l - 1], h->kz[l - 1],
                                 h->kx[l], h->ky[l], h->kz[l]);
            }
        }
    }
    return h;
}

void FN(mg_destroy)(CAT(m2so_mg_, SFX) * h)
{
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) {
        free(h->az[l]);
        free(h->rc[l]);
        free(h->zc[l]);
        free(h->kx[l]);
        free(h->ky[l]);
        free(h->kz[l]);
    }
    free(h);
}

/* Coarse face arrays of level l (VAR7), for tests. */
const REAL *FN(mg_faces)(CAT(m2so_mg_, SFX) * h, int l, int axis)
{
    if (!h || h->kind != 1 || l < 0 || l >= h->nlev) return NULL;
    return axis == 0 ? h->kx[l] : axis == 1 ? h->ky[l] : h->kz[l];
}

/* V-cycle at level l, z = M_l^{-1} r:
 *   z = 0; pre-smooth with one SymGS (forward then backward);
 *   if not coarsest: rc = restrict(r - A z); zc = V-cycle(rc) at l+1;
 *                    z += prolong(zc); post-smooth with one SymGS from the
 *                    current z.
 *   coarsest level: the single SymGS from z = 0 is the whole solve. */
static void CAT(mg_vcycle_l_, SFX)(CAT(m2so_mg_, SFX) * h, int l,
                                   const REAL *r, REAL *z)
{
    long n = (long)h->nx[l] * h->ny[l] * h->nz[l];
    for (long p = 0; p < n; ++p) z[p] = 0;
    CAT(mg_symgs_, SFX)(h, l, r, z);
    if (l == h->nlev - 1) return;
    CAT(mg_apply_, SFX)(h, l, z, h->az[l]);
    FN(restrict_inject)(h->nx[l], h->ny[l], h->nz[l], r, h->az[l],
                        h->rc[l + 1]);
    CAT(mg_vcycle_l_, SFX)(h, l + 1, h->rc[l + 1], h->zc[l + 1]);
    FN(prolong_inject)(h->nx[l], h->ny[l], h->nz[l], h->zc[l + 1], z);
    CAT(mg_symgs_, SFX)(h, l, r, z);
}

void FN(mg_vcycle)(CAT(m2so_mg_, SFX) * h, const REAL *r, REAL *z)
{
    CAT(mg_vcycle_l_, SFX)(h, 0, r, z);
}

#include "m2s_oracle_micro.h"

#undef KX
#undef KY
#undef KZ
#undef IDX
#undef FN
#undef CAT
#undef CAT2
