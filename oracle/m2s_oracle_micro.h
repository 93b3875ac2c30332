/*
 * m2s_oracle_micro.h -- the microbenchmark part of the CPU oracle (Jacobi,
 * the incomplete factorisations of the 27-point operator, the line solves),
 * included by m2s_oracle_impl.h once per floating-point type with its
 * macros (REAL, SFX, FN, CAT, IDX) defined.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of the oracle: loaded only by the
 * test suite, the smoke check and the benchmark's CPU-baseline leg; it
 * shares no code with the library.
 */

/* ------------------------------------------------------------------------
 * Microbenchmarks of Sec. 7.2.1.
 * ---------------------------------------------------------------------- */

/* JacIter: Jacobi iterations of the 2-D 9-point operator on an nx*ny grid
 * ([ny][nx], x fastest): A has `diag` on the diagonal and `off` for each of
 * the up to 8 in-grid neighbours, and one iteration is
 *   x_{t+1}[p] = (b[p] - off * sum_{q in N8(p)} x_t[q]) / diag,
 * the neighbours summed in lexicographic offset order (dy, then dx, each
 * from -1 to +1).  x holds x_0 on entry and x_iters on exit; tmp holds
 * nx*ny values. */
void FN(jacobi9)(int nx, int ny, REAL diag, REAL off, const REAL *b, REAL *x,
                 int iters, REAL *tmp)
{
    for (int t = 0; t < iters; ++t) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                REAL s = 0;
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        const int ii = i + di, jj = j + dj;
                        if ((di == 0 && dj == 0) || ii < 0 || ii >= nx ||
                            jj < 0 || jj >= ny)
                            continue;
                        s += x[(long)jj * nx + ii];
                    }
                tmp[(long)j * nx + i] = (b[(long)j * nx + i] - off * s) / diag;
            }
        memcpy(x, tmp, sizeof(REAL) * (size_t)nx * (size_t)ny);
    }
}

/* D-ILU of the 27-point operator (the factored-diagonal incomplete
 * factorisation: the off-diagonal entries of A kept, only the diagonal
 * factored; not ILU(0), which follows below): M = (D + L) D^{-1} (D + U), L
 * and U the strict lower and upper parts of A and D = diag(d) chosen so that
 * diag(M) = diag(A):
 *   d_p = diag - sum_{q in N27(p), q < p} off * off / d_q,   p ascending,
 * the lower neighbours summed in lexicographic offset order. */
void FN(dilu27_factor)(int nx, int ny, int nz, REAL diag, REAL off, REAL *d)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long p = IDX(i, j, k);
                REAL s = 0;
                for (int dk = -1; dk <= 1; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            const int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny ||
                                kk < 0 || kk >= nz)
                                continue;
                            const long q = IDX(ii, jj, kk);
                            if (q >= p) continue;
                            s += off * off / d[q];
                        }
                d[p] = diag - s;
            }
}

/* z = M^{-1} r with M as above: the lower solve (D + L) y = r, p
 * ascending, y_p = (r_p - off * sum_{q lower} y_q) / d_p; then the upper
 * solve D^{-1} (D + U) z = y, p descending, z_p = y_p - off * (sum_{q upper}
 * z_q) / d_p.  Neighbours summed in lexicographic offset order. */
void FN(dilu27_solve)(int nx, int ny, int nz, REAL off, const REAL *d,
                     const REAL *r, REAL *z)
{
    const long n = (long)nx * ny * nz;
    for (long p = 0; p < n; ++p) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny),
                  k = (int)(p / ((long)nx * ny));
        REAL s = 0;
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                        kk >= nz)
                        continue;
                    const long q = IDX(ii, jj, kk);
                    if (q < p) s += z[q];
                }
        z[p] = (r[p] - off * s) / d[p];
    }
    for (long p = n - 1; p >= 0; --p) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny),
                  k = (int)(p / ((long)nx * ny));
        REAL s = 0;
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                        kk >= nz)
                        continue;
                    const long q = IDX(ii, jj, kk);
                    if (q > p) s += z[q];
                }
        z[p] = z[p] - off * s / d[p];
    }
}

/* ILU(0) of the 27-point operator (the incomplete LU of the ILU
 * microbenchmark, Sec. 7.2.1, as the paper cites it, Sec. 9): L unit lower
 * and U upper triangular with the sparsity pattern of A, computed row by
 * row in lexicographic order by the IKJ form of Gaussian elimination with
 * every fill-in outside the pattern dropped.  For row p, with w the row of A
 * over the 27 offsets, for each lower neighbour q = p + a (offsets in
 * increasing order): l_pq = w_a / u_qq, then w_b -= l_pq u_{q, p+b} for every
 * later offset b of the row whose p + b is an upper neighbour of q; the row
 * of U is what is left of w from the diagonal on.
 * Lf holds per point the 13 entries l_pq of the lower offsets, Uf the pivot
 * u_pp and the 13 entries of the upper offsets (offsets in lexicographic
 * (dk, dj, di) order; 0 outside the grid).  Returns 0, or -1 on a zero
 * pivot. */
static inline int CAT(off27_, SFX)(int m, int *dk, int *dj, int *di)
{
    *dk = m / 9 - 1;
    *dj = (m / 3) % 3 - 1;
    *di = m % 3 - 1;
    return 0;
}

int FN(ilu0_27_factor)(int nx, int ny, int nz, REAL diag, REAL off,
                       REAL *Lf, REAL *Uf)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long p = IDX(i, j, k);
                REAL w[27];
                int in[27];
                for (int m = 0; m < 27; ++m) {
                    int dk, dj, di;
                    CAT(off27_, SFX)(m, &dk, &dj, &di);
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    in[m] = ii >= 0 && ii < nx && jj >= 0 && jj < ny &&
                            kk >= 0 && kk < nz;
                    w[m] = in[m] ? (m == 13 ? diag : off) : (REAL)0;
                }
                for (int a = 0; a < 13; ++a) {
                    if (!in[a]) continue;
                    int ak, aj, ai;
                    CAT(off27_, SFX)(a, &ak, &aj, &ai);
                    const long q = IDX(i + ai, j + aj, k + ak);
                    const REAL l = w[a] / Uf[14 * q];
                    w[a] = l;
                    for (int b = a + 1; b < 27; ++b) {
                        if (!in[b]) continue;
                        int bk, bj, bi;
                        CAT(off27_, SFX)(b, &bk, &bj, &bi);
                        const int ek = bk - ak, ej = bj - aj, ei = bi - ai;
                        if (ek < -1 || ek > 1 || ej < -1 || ej > 1 ||
                            ei < -1 || ei > 1)
                            continue;
                        const int e = 9 * (ek + 1) + 3 * (ej + 1) + (ei + 1);
                        if (e <= 13) continue;  /* not an upper neighbour of q */
                        w[b] -= l * Uf[14 * q + 1 + (e - 14)];
                    }
                }
                if (w[13] == (REAL)0) return -1;
                for (int a = 0; a < 13; ++a) Lf[13 * p + a] = w[a];
                Uf[14 * p] = w[13];
                for (int b = 14; b < 27; ++b) Uf[14 * p + 1 + (b - 14)] = w[b];
            }
    return 0;
}

/* z = (L U)^{-1} r with the factors above: the lower solve L y = r, p
 * ascending, y_p = r_p - sum_{a lower} l_pq y_q; then the upper solve
 * U z = y, p descending, z_p = (y_p - sum_{b upper} u_pq z_q) / u_pp; the
 * offsets summed in lexicographic order. */
void FN(ilu0_27_solve)(int nx, int ny, int nz, const REAL *Lf,
                       const REAL *Uf, const REAL *r, REAL *z)
{
    const long n = (long)nx * ny * nz;
    for (long p = 0; p < n; ++p) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny),
                  k = (int)(p / ((long)nx * ny));
        REAL s = 0;
        for (int a = 0; a < 13; ++a) {
            int dk, dj, di;
            CAT(off27_, SFX)(a, &dk, &dj, &di);
            const int ii = i + di, jj = j + dj, kk = k + dk;
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                kk >= nz)
                continue;
            s += Lf[13 * p + a] * z[IDX(ii, jj, kk)];
        }
        z[p] = r[p] - s;
    }
    for (long p = n - 1; p >= 0; --p) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny),
                  k = (int)(p / ((long)nx * ny));
        REAL s = 0;
        for (int b = 14; b < 27; ++b) {
            int dk, dj, di;
            CAT(off27_, SFX)(b, &dk, &dj, &di);
            const int ii = i + di, jj = j + dj, kk = k + dk;
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 ||
                kk >= nz)
                continue;
            s += Uf[14 * p + 1 + (b - 14)] * z[IDX(ii, jj, kk)];
        }
        z[p] = (z[p] - s) / Uf[14 * p];
    }
}

/* Pentadiagonal line solves (the scalar multi-diagonal systems of the ADI-
 * shaped NPB SP solver, Sec. 7.1): along axis `dir` (0 x, 1 y, 2 z) every
 * grid line holds the system
 *   a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2} = r_i
 * (i the position on the line; terms reaching off the line are absent),
 * coef = [5][nz][ny][nx] holding a, b, c, d, e at every point.  Each line is
 * solved by Gaussian elimination without pivoting: eliminate the two
 * sub-diagonals row by row from the top, then substitute back from the
 * bottom. */
void FN(penta_lines)(int nx, int ny, int nz, int dir, const REAL *coef,
                     const REAL *r, REAL *x)
{
    const long n = (long)nx * ny * nz;
    const int len = dir == 0 ? nx : dir == 1 ? ny : nz;
    const long stride = dir == 0 ? 1 : dir == 1 ? nx : (long)nx * ny;
    REAL *w = (REAL *)malloc(sizeof(REAL) * 4 * (size_t)len);  /* c d e r */
    for (long base = 0; base < n; ++base) {
        const int i0 = (int)(base % nx), j0 = (int)((base / nx) % ny),
                  k0 = (int)(base / ((long)nx * ny));
        if ((dir == 0 && i0) || (dir == 1 && j0) || (dir == 2 && k0))
            continue;  /* base is the first point of its line */
        REAL *C = w, *D = w + len, *E = w + 2 * len, *R = w + 3 * len;
        for (int i = 0; i < len; ++i) {
            const long p = base + i * stride;
            C[i] = coef[2 * n + p];
            D[i] = coef[3 * n + p];
            E[i] = coef[4 * n + p];
            R[i] = r[p];
        }
        for (int i = 0; i < len; ++i) {
            const long p = base + i * stride;
            /* row i still holds its own a_i, b_i; remove x_{i-2}, x_{i-1} */
            REAL a = coef[0 * n + p], b = coef[1 * n + p];
            if (i >= 2) {
                const REAL f = a / C[i - 2];
                b -= f * D[i - 2];
                C[i] -= f * E[i - 2];
                R[i] -= f * R[i - 2];
            }
            if (i >= 1) {
                const REAL f = b / C[i - 1];
                C[i] -= f * D[i - 1];
                D[i] -= f * E[i - 1];
                R[i] -= f * R[i - 1];
            }
        }
        for (int i = len - 1; i >= 0; --i) {
            REAL v = R[i];
            if (i + 1 < len) v -= D[i] * x[base + (i + 1) * stride];
            if (i + 2 < len) v -= E[i] * x[base + (i + 2) * stride];
            x[base + i * stride] = v / C[i];
        }
    }
    free(w);
}

/* Solve M X = Y for a 5x5 matrix M and a 5 x ncol right-hand side Y (both
 * row-major; Y is overwritten by X, M by its elimination) by Gaussian
 * elimination with partial pivoting.  Returns 0, or -1 if a pivot is 0. */
static int FN(solve5)(REAL *M, REAL *Y, int ncol)
{
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int q = c + 1; q < 5; ++q)
            if (fabs((double)M[q * 5 + c]) > fabs((double)M[piv * 5 + c]))
                piv = q;
        if (M[piv * 5 + c] == 0) return -1;
        if (piv != c) {
            for (int k = 0; k < 5; ++k) {
                const REAL t = M[c * 5 + k];
                M[c * 5 + k] = M[piv * 5 + k];
                M[piv * 5 + k] = t;
            }
            for (int k = 0; k < ncol; ++k) {
                const REAL t = Y[c * ncol + k];
                Y[c * ncol + k] = Y[piv * ncol + k];
                Y[piv * ncol + k] = t;
            }
        }
        for (int q = c + 1; q < 5; ++q) {
            const REAL f = M[q * 5 + c] / M[c * 5 + c];
            for (int k = c; k < 5; ++k) M[q * 5 + k] -= f * M[c * 5 + k];
            for (int k = 0; k < ncol; ++k) Y[q * ncol + k] -= f * Y[c * ncol + k];
        }
    }
    for (int c = 4; c >= 0; --c)
        for (int k = 0; k < ncol; ++k) {
            REAL v = Y[c * ncol + k];
            for (int q = c + 1; q < 5; ++q) v -= M[c * 5 + q] * Y[q * ncol + k];
            Y[c * ncol + k] = v / M[c * 5 + c];
        }
    return 0;
}

/* Block-tridiagonal line solves (the 5x5 block systems of the ADI-shaped
 * NPB BT solver, Sec. 7.1): along axis `dir` (0 x, 1 y, 2 z) every grid
 * line holds the system
 *   A_i x_{i-1} + B_i x_i + C_i x_{i+1} = r_i
 * in 5-vectors x_i, r_i and 5x5 blocks (i the position on the line; terms
 * reaching off the line are absent).  coef = [3][nz][ny][nx][5][5] holds
 * A, B, C at every point (row-major blocks); r, x = [nz][ny][nx][5].
 * Block Gaussian elimination down the line, then back substitution (the
 * block Thomas algorithm): with G_{-1} = 0 and y_{-1} = 0,
 *   M_i = B_i - A_i G_{i-1},  G_i = M_i^{-1} C_i,
 *   y_i = M_i^{-1} (r_i - A_i y_{i-1});
 *   x_{L-1} = y_{L-1},  x_i = y_i - G_i x_{i+1}.
 * Returns 0, or -1 if some M_i is singular. */
int FN(bt_lines)(int nx, int ny, int nz, int dir, const REAL *coef,
                 const REAL *r, REAL *x)
{
    const long n = (long)nx * ny * nz;
    const int len = dir == 0 ? nx : dir == 1 ? ny : nz;
    const long stride = dir == 0 ? 1 : dir == 1 ? nx : (long)nx * ny;
    REAL *G = (REAL *)malloc(sizeof(REAL) * 25 * (size_t)len);
    REAL *Yv = (REAL *)malloc(sizeof(REAL) * 5 * (size_t)len);
    int status = 0;
    for (long base = 0; base < n && status == 0; ++base) {
        const int i0 = (int)(base % nx), j0 = (int)((base / nx) % ny),
                  k0 = (int)(base / ((long)nx * ny));
        if ((dir == 0 && i0) || (dir == 1 && j0) || (dir == 2 && k0))
            continue;  /* base is the first point of its line */
        for (int i = 0; i < len; ++i) {
            const long p = base + i * stride;
            const REAL *A = coef + 25 * p;
            const REAL *B = coef + 25 * (n + p);
            const REAL *Cb = coef + 25 * (2 * n + p);
            /* the augmented system [M | C_i  r_i - A_i y_{i-1}] */
            REAL M[25], Y[30];
            for (int a = 0; a < 5; ++a) {
                for (int b = 0; b < 5; ++b) {
                    REAL m = B[a * 5 + b];
                    if (i > 0)
                        for (int c = 0; c < 5; ++c)
                            m -= A[a * 5 + c] * G[25 * (i - 1) + c * 5 + b];
                    M[a * 5 + b] = m;
                    Y[a * 6 + b] = Cb[a * 5 + b];
                }
                REAL v = r[5 * p + a];
                if (i > 0)
                    for (int c = 0; c < 5; ++c)
                        v -= A[a * 5 + c] * Yv[5 * (i - 1) + c];
                Y[a * 6 + 5] = v;
            }
            if (FN(solve5)(M, Y, 6)) {
                status = -1;
                break;
            }
            for (int a = 0; a < 5; ++a) {
                for (int b = 0; b < 5; ++b) G[25 * i + a * 5 + b] = Y[a * 6 + b];
                Yv[5 * i + a] = Y[a * 6 + 5];
            }
        }
        if (status) break;
        for (int i = len - 1; i >= 0; --i) {
            const long p = base + i * stride;
            for (int a = 0; a < 5; ++a) {
                REAL v = Yv[5 * i + a];
                if (i + 1 < len)
                    for (int c = 0; c < 5; ++c)
                        v -= G[25 * i + a * 5 + c] *
                             x[5 * (base + (i + 1) * stride) + c];
                x[5 * p + a] = v;
            }
        }
    }
    free(G);
    free(Yv);
    return status;
}

