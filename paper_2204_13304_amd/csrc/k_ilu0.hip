// k_ilu0.hip -- ILU(0) of the 27-point operator (the incomplete LU of the
// ILU microbenchmark, Sec. 7.2.1, as cited in Sec. 9): the factorisation
// and the two triangular solves, scheduled by hyperplanes.
//
// The factor of row p needs the finished U rows of its 13 lower
// neighbours, the lower solve their y values, the upper solve the z values
// of its 13 upper neighbours: the dependence pattern of the Gauss-Seidel
// sweep, so point (i, j, k) runs at step T = i + 2j + 4k (Eq.
// (hyperplane), Sec. 6.1.3; weights (1, 2, 4) legal for the 27 points) and
// every point of a step is independent.  One launch per step, one thread
// per point of the step; the upper solve walks the steps backwards.  Each
// row carries 27 coefficients (13 of L, 14 of U), so unlike the
// constant-coefficient sweeps these passes are bound by reading the
// factors, and a point's whole row stays in registers.
//
// Factor arrays, per point p in C order of (nz, ny, nx): L[13 p + a] =
// l_pq for the lower offsets a = 0..12, U[14 p] = u_pp and U[14 p + 1 + b]
// = u_pq for the upper offsets b = 0..12; offsets in lexicographic
// (dk, dj, di) order, 0 for neighbours outside the grid.
#include "m2s_internal.hpp"

namespace m2s {

namespace {

__device__ __forceinline__ void off27(int m, int &dk, int &dj, int &di)
{
    dk = m / 9 - 1;
    dj = (m / 3) % 3 - 1;
    di = m % 3 - 1;
}

// point of step T handled by this thread: (j, k) from the launch grid, i
// from T; false when outside the grid
__device__ __forceinline__ bool step_point(const Grid &g, int T, int k0,
                                           int &i, int &j, int &k)
{
    j = blockIdx.x * blockDim.x + threadIdx.x;
    k = k0 + blockIdx.y;
    if (j >= g.ny || k >= g.nz) return false;
    i = T - 2 * j - 4 * k;
    return i >= 0 && i < g.nx;
}

// Row p of the IKJ elimination with the fill outside A's pattern dropped:
// w = row p of A; for each lower neighbour q = p + a in offset order,
// l = w_a / u_qq, then w_b -= l u_{q, p+b} for the later offsets b whose
// p + b is an upper neighbour of q.  The order of the operations is the
// definition's, so the factor equals the CPU oracle's bit for bit.
__global__ void __launch_bounds__(256)
    ilu0_factor_kernel(Grid g, double diag, double off, int T, int k0,
                       double *__restrict__ L, double *__restrict__ U)
{
    int i, j, k;
    if (!step_point(g, T, k0, i, j, k)) return;
    const int64_t p = g.idx(i, j, k);
    double w[27];
    bool in[27];
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        int dk, dj, di;
        off27(m, dk, dj, di);
        in[m] = g.in(i + di, j + dj, k + dk);
        w[m] = in[m] ? (m == 13 ? diag : off) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 13; ++a) {
        if (!in[a]) continue;
        int ak, aj, ai;
        off27(a, ak, aj, ai);
        const int64_t q = g.idx(i + ai, j + aj, k + ak);
        const double *Uq = U + 14 * q;
        const double l = w[a] / Uq[0];
        w[a] = l;
#pragma unroll
        for (int b = a + 1; b < 27; ++b) {
            int bk, bj, bi;
            off27(b, bk, bj, bi);
            const int ek = bk - ak, ej = bj - aj, ei = bi - ai;
            if (ek < -1 || ek > 1 || ej < -1 || ej > 1 || ei < -1 || ei > 1)
                continue;
            const int e = 9 * (ek + 1) + 3 * (ej + 1) + (ei + 1);
            if (e <= 13 || !in[b]) continue;
            w[b] -= l * Uq[1 + (e - 14)];
        }
    }
#pragma unroll
    for (int a = 0; a < 13; ++a) L[13 * p + a] = w[a];
    U[14 * p] = w[13];
#pragma unroll
    for (int b = 14; b < 27; ++b) U[14 * p + 1 + (b - 14)] = w[b];
}

// Lower solve L y = r at step T: y_p = r_p - sum_a l_pq y_q, offsets in
// order (y written into out).
__global__ void __launch_bounds__(256)
    ilu0_lower_kernel(Grid g, int T, int k0, const double *__restrict__ L,
                      const double *__restrict__ r, double *__restrict__ y)
{
    int i, j, k;
    if (!step_point(g, T, k0, i, j, k)) return;
    const int64_t p = g.idx(i, j, k);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 13; ++a) {
        int dk, dj, di;
        off27(a, dk, dj, di);
        if (!g.in(i + di, j + dj, k + dk)) continue;
        s += L[13 * p + a] * y[g.idx(i + di, j + dj, k + dk)];
    }
    y[p] = r[p] - s;
}

// Upper solve U z = y at step T, in place on z (which holds y): z_p =
// (y_p - sum_b u_pq z_q) / u_pp, offsets in order.
__global__ void __launch_bounds__(256)
    ilu0_upper_kernel(Grid g, int T, int k0, const double *__restrict__ U,
                      double *__restrict__ z)
{
    int i, j, k;
    if (!step_point(g, T, k0, i, j, k)) return;
    const int64_t p = g.idx(i, j, k);
    double s = 0.0;
#pragma unroll
    for (int b = 14; b < 27; ++b) {
        int dk, dj, di;
        off27(b, dk, dj, di);
        if (!g.in(i + di, j + dj, k + dk)) continue;
        s += U[14 * p + 1 + (b - 14)] * z[g.idx(i + di, j + dj, k + dk)];
    }
    z[p] = (z[p] - s) / U[14 * p];
}

// launch geometry of step T: the planes k with a point on it (0 <= T - 2j -
// 4k < nx for some 0 <= j < ny), one thread per j
struct StepLaunch {
    dim3 grid, block;
    int k0;
    bool empty;
};

StepLaunch step_launch(const Grid &g, int T)
{
    StepLaunch s{};
    const int kmin = std::max(0, (T - (g.nx - 1) - 2 * (g.ny - 1) + 3) / 4);
    const int kmax = std::min(g.nz - 1, T / 4);
    s.empty = kmin > kmax;
    s.k0 = kmin;
    const int bx = std::min(256, ((g.ny + 63) / 64) * 64);
    s.block = dim3(bx);
    s.grid = dim3((g.ny + bx - 1) / bx, s.empty ? 1 : kmax - kmin + 1);
    return s;
}

int n_steps(const Grid &g)
{
    return (g.nx - 1) + 2 * (g.ny - 1) + 4 * (g.nz - 1) + 1;
}

}  // namespace

hipError_t launch_ilu0_factor(const m2s_stencil &A, double *L, double *U,
                              hipStream_t s)
{
    const Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    for (int T = 0; T < n_steps(g); ++T) {
        const StepLaunch sl = step_launch(g, T);
        if (sl.empty) continue;
        hipLaunchKernelGGL(ilu0_factor_kernel, sl.grid, sl.block, 0, s, g,
                           A.diag, A.offdiag, T, sl.k0, L, U);
    }
    return hipGetLastError();
}

hipError_t launch_ilu0_apply(const m2s_stencil &A, const double *L,
                             const double *U, const double *r, double *z,
                             hipStream_t s)
{
    const Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int H = n_steps(g);
    for (int T = 0; T < H; ++T) {
        const StepLaunch sl = step_launch(g, T);
        if (sl.empty) continue;
        hipLaunchKernelGGL(ilu0_lower_kernel, sl.grid, sl.block, 0, s, g, T,
                           sl.k0, L, r, z);
    }
    for (int T = H - 1; T >= 0; --T) {
        const StepLaunch sl = step_launch(g, T);
        if (sl.empty) continue;
        hipLaunchKernelGGL(ilu0_upper_kernel, sl.grid, sl.block, 0, s, g, T,
                           sl.k0, U, z);
    }
    return hipGetLastError();
}

}  // namespace m2s
