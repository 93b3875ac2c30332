// k_lines.hip -- batched pentadiagonal line solves (the scalar multi-
// diagonal systems of the ADI-shaped NPB SP solver, Sec. 7.1) for gfx950.
//
// Along axis x, y or z every grid line holds the system
//   a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2} = r_i.
// Each line is a sequential (Seidel-style, 1-D) recurrence, the lines are
// independent: one thread per line runs the forward elimination and then
// the back substitution (fused, one launch).  The elimination keeps the
// rows normalised -- row i becomes x_i + u_i x_{i+1} + v_i x_{i+2} = y_i --
// so only u, v (work buffer) and y (kept in x) are stored for the way back:
//   forward  reads a..e, r, writes u, v, y     (72 B per point)
//   backward reads u, v, y, writes x           (32 B per point).
// Threads next to each other take lines next to each other: for y and z
// lines those are neighbouring x positions, so every access is coalesced;
// x lines are contiguous per thread.  Loads run ahead of the recurrence
// (the coefficients do not depend on it).
#include "m2s_internal.hpp"

namespace m2s {

constexpr int PL_NT = 64;

__global__ void __launch_bounds__(PL_NT)
    penta_lines_kernel(int nx, int ny, int nz, int axis,
                       const double *__restrict__ coef,
                       const double *__restrict__ r, double *__restrict__ x,
                       double *__restrict__ work)
{
    const long n = (long)nx * ny * nz;
    const int line = blockIdx.x * PL_NT + threadIdx.x;
    long base, stride;
    int len, nlines;
    if (axis == 0) {
        nlines = ny * nz;
        base = (long)line * nx;
        stride = 1;
        len = nx;
    } else if (axis == 1) {
        nlines = nx * nz;
        const int i = line % nx, k = line / nx;
        base = (long)k * nx * ny + i;
        stride = nx;
        len = ny;
    } else {
        nlines = nx * ny;
        base = line;
        stride = (long)nx * ny;
        len = nz;
    }
    if (line >= nlines) return;
    const double *ca = coef, *cb = coef + n, *cc = coef + 2 * n,
                 *cd = coef + 3 * n, *ce = coef + 4 * n;
    double *u = work, *v = work + n;

    // forward elimination; (u1, v1, y1) row i - 1, (u2, v2, y2) row i - 2
    double u1 = 0, v1 = 0, y1 = 0, u2 = 0, v2 = 0, y2 = 0;
    long p = base;
#pragma unroll 4
    for (int i = 0; i < len; ++i, p += stride) {
        const double a = i >= 2 ? ca[p] : 0.0;
        double bb = i >= 1 ? cb[p] : 0.0;
        double c = cc[p], d = cd[p];
        const double e = ce[p];
        double rr = r[p];
        // remove x_{i-2} with row i - 2, then x_{i-1} with row i - 1
        bb -= a * u2;
        c -= a * v2;
        rr -= a * y2;
        c -= bb * u1;
        d -= bb * v1;
        rr -= bb * y1;
        const double inv = 1.0 / c;
        const double ui = d * inv, vi = e * inv, yi = rr * inv;
        u[p] = ui;
        v[p] = vi;
        x[p] = yi;
        u2 = u1;
        v2 = v1;
        y2 = y1;
        u1 = ui;
        v1 = vi;
        y1 = yi;
    }
    // back substitution: x_i = y_i - u_i x_{i+1} - v_i x_{i+2}
    double x1 = 0, x2 = 0;
    p = base + (long)(len - 1) * stride;
#pragma unroll 4
    for (int i = len - 1; i >= 0; --i, p -= stride) {
        const double xi = x[p] - u[p] * x1 - v[p] * x2;
        x[p] = xi;
        x2 = x1;
        x1 = xi;
    }
}

hipError_t launch_penta_lines(int nx, int ny, int nz, int axis,
                              const double *coef, const double *r, double *x,
                              double *work, hipStream_t s)
{
    const long nlines = axis == 0   ? (long)ny * nz
                        : axis == 1 ? (long)nx * nz
                                    : (long)nx * ny;
    const int grid = (int)((nlines + PL_NT - 1) / PL_NT);
    hipLaunchKernelGGL(penta_lines_kernel, dim3(grid), dim3(PL_NT), 0, s, nx,
                       ny, nz, axis, coef, r, x, work);
    return hipGetLastError();
}

}  // namespace m2s
