// k_lines.hip -- batched line solves for gfx950: pentadiagonal (the scalar
// multi-diagonal systems of the ADI-shaped NPB SP solver, Sec. 7.1) and
// 5x5 block-tridiagonal (those of NPB BT; at the end of the file).
//
// Along axis x, y or z every grid line holds the system
//   a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2} = r_i.
// Each line is a sequential (Seidel-style, 1-D) recurrence, the lines are
// independent: one lane per line runs the forward elimination and then the
// back substitution (fused, one launch).  The elimination keeps the rows
// normalised -- row i becomes x_i + u_i x_{i+1} + v_i x_{i+2} = y_i -- so
// only u, v (work buffer) and y (kept in x) are stored for the way back:
//   forward  reads a..e, r, writes u, v, y     (72 B per point)
//   backward reads u, v, y, writes x           (32 B per point).
//
// A 64-lane workgroup takes LW = 64 / S lines and walks them in chunks of
// 8 S points staged through LDS: the whole workgroup loads a chunk of every
// input array with coalesced accesses (runs along x for x lines, the lines'
// neighbouring x positions for y and z lines), lanes 0 .. LW - 1 run the
// recurrence over their line's chunk in LDS, and the chunk's outputs leave
// through LDS with coalesced stores.  The next chunk's loads are in flight
// (in registers) while the current chunk is computed.  With only n^2 lines
// the solve is bound by the loads in flight per line, not by arithmetic:
// S lanes per line in the transfers multiply them (and the workgroups) by S
// at the same register count per lane.
#include "m2s_internal.hpp"

#include <cstdlib>

namespace m2s {

constexpr int PL_NT = 64;   // lanes per workgroup
constexpr int PL_M = 8;     // transfer elements per lane per array and chunk

// LDS row stride (doubles) for S lanes per line: a pass of 16 lanes hits 16
// distinct 8-byte banks in the x-line transfers (S = 1: 8 points of 2 lines,
// stride 2 mod 16; S > 1: 16 points of one line, odd stride), in the y- and
// z-line transfers and in the compute loop (consecutive lines).
template <int S>
constexpr int pl_ls() { return S == 1 ? 66 : PL_NT / S + 1; }

template <int AXIS>
struct LineMap {
    int nx, ny, nz;
    __device__ int nlines() const
    {
        return AXIS == 0 ? ny * nz : AXIS == 1 ? nx * nz : nx * ny;
    }
    __device__ int len() const { return AXIS == 0 ? nx : AXIS == 1 ? ny : nz; }
    __device__ long stride() const
    {
        return AXIS == 0 ? 1 : AXIS == 1 ? (long)nx : (long)nx * ny;
    }
    __device__ long base(int line) const
    {
        if (AXIS == 0) return (long)line * nx;
        if (AXIS == 1) {
            const int k = line / nx, i = line - k * nx;
            return (long)k * nx * ny + i;
        }
        return line;
    }
};

// Element m of a lane's share of a chunk transfer: (line l, point q) of the
// chunk.  x lines: consecutive lanes cover consecutive points of a line
// (runs of 8 S values); y and z lines: consecutive lanes cover the lines.
template <int AXIS, int S>
__device__ __forceinline__ void chunk_elem(int t, int m, int &l, int &q)
{
    constexpr int LW = PL_NT / S, CHS = PL_M * S;
    const int e = t + PL_NT * m;
    if (AXIS == 0) {
        l = e / CHS;
        q = e - l * CHS;
    } else {
        l = e % LW;
        q = e / LW;
    }
}

template <int AXIS, int S>
__global__ void __launch_bounds__(PL_NT)
    penta_lines_kernel(int nx, int ny, int nz, const double *__restrict__ coef,
                       const double *__restrict__ r, double *__restrict__ x,
                       double *__restrict__ work)
{
    constexpr int LW = PL_NT / S, CHS = PL_M * S, LS = pl_ls<S>();
    __shared__ double sm[6][CHS * LS];
    const LineMap<AXIS> M{nx, ny, nz};
    const long n = (long)nx * ny * nz;
    const int nl = M.nlines(), len = M.len();
    const long st = M.stride();
    const int t = threadIdx.x;
    const int L0 = blockIdx.x * LW;
    const int nch = (len + CHS - 1) / CHS;
    const bool runs = t < LW;  // this lane runs line L0 + t
    double *const u = work, *const v = work + n;

    // the lane's transfer elements: global base of their lines, point slots
    long gb[PL_M];
    int lq[PL_M], qq[PL_M];
    bool lv[PL_M];
#pragma unroll
    for (int m = 0; m < PL_M; ++m) {
        int l, q;
        chunk_elem<AXIS, S>(t, m, l, q);
        lv[m] = L0 + l < nl;
        gb[m] = lv[m] ? M.base(L0 + l) : 0;
        lq[m] = q * LS + l;
        qq[m] = q;
    }
    auto gaddr = [&](int m, int c) {
        return gb[m] + (long)(c * CHS + qq[m]) * st;
    };
    auto in_range = [&](int m, int c) {
        return lv[m] && c * CHS + qq[m] < len;
    };

    // ---- forward elimination, chunks in increasing order
    double pre[6][PL_M];
    auto fetch_fwd = [&](int c) {
#pragma unroll
        for (int m = 0; m < PL_M; ++m) {
            const bool ok = in_range(m, c);
            const long g = ok ? gaddr(m, c) : 0;
#pragma unroll
            for (int a = 0; a < 5; ++a)
                pre[a][m] = ok ? coef[a * n + g] : (a == 2 ? 1.0 : 0.0);
            pre[5][m] = ok ? r[g] : 0.0;
        }
    };
    double u1 = 0, v1 = 0, y1 = 0, u2 = 0, v2 = 0, y2 = 0;
    fetch_fwd(0);
    for (int c = 0; c < nch; ++c) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PL_M; ++m)
#pragma unroll
            for (int a = 0; a < 6; ++a) sm[a][lq[m]] = pre[a][m];
        __syncthreads();
        if (c + 1 < nch) fetch_fwd(c + 1);
        // the lane's own line: row q of the chunk at sm[.][q * LS + t]
        if (runs) {
#pragma unroll 4
            for (int q = 0; q < CHS; ++q) {
                const int i = c * CHS + q;
                const int o = q * LS + t;
                const double a = i >= 2 ? sm[0][o] : 0.0;
                double bb = i >= 1 ? sm[1][o] : 0.0;
                double cc = sm[2][o], d = sm[3][o];
                const double e = sm[4][o];
                double rr = sm[5][o];
                // remove x_{i-2} with row i - 2, then x_{i-1} with row i - 1
                bb -= a * u2;
                cc -= a * v2;
                rr -= a * y2;
                cc -= bb * u1;
                d -= bb * v1;
                rr -= bb * y1;
                const double inv = 1.0 / cc;
                const double ui = d * inv, vi = e * inv, yi = rr * inv;
                sm[0][o] = ui;
                sm[1][o] = vi;
                sm[2][o] = yi;
                u2 = u1;
                v2 = v1;
                y2 = y1;
                u1 = ui;
                v1 = vi;
                y1 = yi;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PL_M; ++m)
            if (in_range(m, c)) {
                const long g = gaddr(m, c);
                u[g] = sm[0][lq[m]];
                v[g] = sm[1][lq[m]];
                x[g] = sm[2][lq[m]];
            }
    }

    // ---- back substitution, chunks in decreasing order.  Transfers map
    // elements to lanes the same way in both passes, so each lane loads back
    // exactly the u, v, y values it stored itself.
    auto fetch_bwd = [&](int c) {
#pragma unroll
        for (int m = 0; m < PL_M; ++m) {
            const bool ok = in_range(m, c);
            const long g = ok ? gaddr(m, c) : 0;
            pre[0][m] = ok ? u[g] : 0.0;
            pre[1][m] = ok ? v[g] : 0.0;
            pre[2][m] = ok ? x[g] : 0.0;
        }
    };
    double x1 = 0, x2 = 0;
    fetch_bwd(nch - 1);
    for (int c = nch - 1; c >= 0; --c) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PL_M; ++m)
#pragma unroll
            for (int a = 0; a < 3; ++a) sm[a][lq[m]] = pre[a][m];
        __syncthreads();
        if (c > 0) fetch_bwd(c - 1);
        if (runs) {
#pragma unroll 4
            for (int q = CHS - 1; q >= 0; --q) {
                const int i = c * CHS + q;
                const int o = q * LS + t;
                if (i < len) {
                    // x_i = y_i - u_i x_{i+1} - v_i x_{i+2}
                    const double xi =
                        sm[2][o] - sm[0][o] * x1 - sm[1][o] * x2;
                    sm[2][o] = xi;
                    x2 = x1;
                    x1 = xi;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PL_M; ++m)
            if (in_range(m, c)) x[gaddr(m, c)] = sm[2][lq[m]];
    }
}

template <int S>
static hipError_t penta_launch(int nx, int ny, int nz, int axis,
                               const double *coef, const double *r,
                               double *x, double *work, hipStream_t s)
{
    constexpr int LW = PL_NT / S;
    const long nlines = axis == 0   ? (long)ny * nz
                        : axis == 1 ? (long)nx * nz
                                    : (long)nx * ny;
    const int grid = (int)((nlines + LW - 1) / LW);
    auto k = axis == 0   ? penta_lines_kernel<0, S>
             : axis == 1 ? penta_lines_kernel<1, S>
                         : penta_lines_kernel<2, S>;
    hipLaunchKernelGGL(k, dim3(grid), dim3(PL_NT), 0, s, nx, ny, nz, coef, r,
                       x, work);
    return hipGetLastError();
}

hipError_t launch_penta_lines(int nx, int ny, int nz, int axis,
                              const double *coef, const double *r, double *x,
                              double *work, hipStream_t s)
{
    // lanes per line in the transfers (tuning knob; 1, 2 or 4)
    const char *e = getenv("M2S_PL_SPLIT");
    const int split = e ? atoi(e) : 2;
    if (split == 1)
        return penta_launch<1>(nx, ny, nz, axis, coef, r, x, work, s);
    if (split == 4)
        return penta_launch<4>(nx, ny, nz, axis, coef, r, x, work, s);
    return penta_launch<2>(nx, ny, nz, axis, coef, r, x, work, s);
}

// ------------------------------------------------------------------------
// 5x5 block-tridiagonal line solves (the block systems of the ADI-shaped NPB
// BT solver, Sec. 7.1).  Along the axis every line holds
//   A_i x_{i-1} + B_i x_i + C_i x_{i+1} = r_i
// in 5-vectors; coef = [3][n][5][5] (A, B, C per point, row-major), r and x
// = [n][5].  Block elimination down the line keeps G_i = M_i^{-1} C_i and
// y_i = M_i^{-1} (r_i - A_i y_{i-1}) with M_i = B_i - A_i G_{i-1}, then back
// substitution x_i = y_i - G_i x_{i+1}: G goes to the work buffer
// (25 doubles per point), y into x.  One lane per line holds G_{i-1},
// y_{i-1}, the pivot block and its LU in registers; elimination and back
// substitution run in one launch.  The pivot blocks are factored without
// pivoting (the systems must keep them safely nonsingular, e.g. block
// diagonal dominance).
constexpr int BT_NT = 64;

// in-place LU of a 5x5 block without pivoting: unit lower factor below the
// diagonal (the multipliers), upper factor on and above it
__device__ __forceinline__ void bt_lu5(double (&m)[25])
{
#pragma unroll
    for (int c = 0; c < 5; ++c) {
#pragma unroll
        for (int q = c + 1; q < 5; ++q) {
            const double f = m[q * 5 + c] / m[c * 5 + c];
            m[q * 5 + c] = f;
#pragma unroll
            for (int k = c + 1; k < 5; ++k) m[q * 5 + k] -= f * m[c * 5 + k];
        }
    }
}

// v <- M^{-1} v with M's LU from bt_lu5
__device__ __forceinline__ void bt_lu5_solve(const double (&m)[25],
                                             double (&v)[5])
{
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
        for (int q = c + 1; q < 5; ++q) v[q] -= m[q * 5 + c] * v[c];
#pragma unroll
    for (int c = 4; c >= 0; --c) {
#pragma unroll
        for (int q = c + 1; q < 5; ++q) v[c] -= m[c * 5 + q] * v[q];
        v[c] = v[c] / m[c * 5 + c];
    }
}

template <int AXIS>
__global__ void __launch_bounds__(BT_NT)
    bt_lines_kernel(int nx, int ny, int nz, const double *__restrict__ coef,
                    const double *__restrict__ r, double *__restrict__ x,
                    double *__restrict__ work)
{
    const LineMap<AXIS> M{nx, ny, nz};
    const int line = blockIdx.x * BT_NT + threadIdx.x;
    if (line >= M.nlines()) return;
    const long n = (long)nx * ny * nz;
    const int len = M.len();
    const long st = M.stride(), base = M.base(line);

    // ---- elimination down the line.  The next point's blocks and r are
    // loaded into registers while the current point is eliminated, so each
    // lane keeps a point's worth of loads in flight behind its arithmetic.
    double na[25], nb[25], nc[25], nr[5];
    auto fetch = [&](int i) {
        const long p = base + (long)i * st;
        // the first point's A and the last point's C couple to nothing and
        // are not read
        if (i > 0) {
#pragma unroll
            for (int e = 0; e < 25; ++e) na[e] = coef[25 * p + e];
        }
#pragma unroll
        for (int e = 0; e < 25; ++e) nb[e] = coef[25 * (n + p) + e];
        if (i + 1 < len) {
#pragma unroll
            for (int e = 0; e < 25; ++e) nc[e] = coef[25 * (2 * n + p) + e];
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) nr[a] = r[5 * p + a];
    };
    double g[25], y[5];  // G_{i-1}, y_{i-1}
    fetch(0);
    for (int i = 0; i < len; ++i) {
        const long p = base + (long)i * st;
        double ab[25], m[25], cb[25], v[5];
#pragma unroll
        for (int e = 0; e < 25; ++e) {
            ab[e] = na[e];
            m[e] = nb[e];
            cb[e] = nc[e];
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) v[a] = nr[a];
        if (i + 1 < len) fetch(i + 1);
        if (i > 0) {
            // M = B - A G_{i-1}, v = r - A y_{i-1}
#pragma unroll
            for (int a = 0; a < 5; ++a) {
#pragma unroll
                for (int b = 0; b < 5; ++b)
#pragma unroll
                    for (int c = 0; c < 5; ++c)
                        m[a * 5 + b] -= ab[a * 5 + c] * g[c * 5 + b];
#pragma unroll
                for (int c = 0; c < 5; ++c) v[a] -= ab[a * 5 + c] * y[c];
            }
        }
        bt_lu5(m);
        if (i + 1 < len) {
            // G_i = M^{-1} C_i column by column
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                double col[5];
#pragma unroll
                for (int a = 0; a < 5; ++a) col[a] = cb[a * 5 + b];
                bt_lu5_solve(m, col);
#pragma unroll
                for (int a = 0; a < 5; ++a) g[a * 5 + b] = col[a];
            }
#pragma unroll
            for (int e = 0; e < 25; ++e) work[25 * p + e] = g[e];
        }
        bt_lu5_solve(m, v);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            y[a] = v[a];
            x[5 * p + a] = v[a];
        }
    }

    // ---- back substitution: x_{L-1} = y_{L-1} is in place already; the
    // next (lower) point's G and y are loaded while the current one is done
    double xn[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) xn[a] = y[a];
    double ng[25], ny5[5];
    auto fetch_back = [&](int i) {
        const long p = base + (long)i * st;
#pragma unroll
        for (int e = 0; e < 25; ++e) ng[e] = work[25 * p + e];
#pragma unroll
        for (int a = 0; a < 5; ++a) ny5[a] = x[5 * p + a];
    };
    if (len >= 2) fetch_back(len - 2);
    for (int i = len - 2; i >= 0; --i) {
        const long p = base + (long)i * st;
        double gi[25], yi[5], xi[5];
#pragma unroll
        for (int e = 0; e < 25; ++e) gi[e] = ng[e];
#pragma unroll
        for (int a = 0; a < 5; ++a) yi[a] = ny5[a];
        if (i > 0) fetch_back(i - 1);
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            double v = yi[a];
#pragma unroll
            for (int c = 0; c < 5; ++c) v -= gi[a * 5 + c] * xn[c];
            xi[a] = v;
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            x[5 * p + a] = xi[a];
            xn[a] = xi[a];
        }
    }
}

hipError_t launch_bt_lines(int nx, int ny, int nz, int axis,
                           const double *coef, const double *r, double *x,
                           double *work, hipStream_t s)
{
    const long nlines = axis == 0   ? (long)ny * nz
                        : axis == 1 ? (long)nx * nz
                                    : (long)nx * ny;
    const int grid = (int)((nlines + BT_NT - 1) / BT_NT);
    auto k = axis == 0   ? bt_lines_kernel<0>
             : axis == 1 ? bt_lines_kernel<1>
                         : bt_lines_kernel<2>;
    hipLaunchKernelGGL(k, dim3(grid), dim3(BT_NT), 0, s, nx, ny, nz, coef, r,
                       x, work);
    return hipGetLastError();
}

}  // namespace m2s
