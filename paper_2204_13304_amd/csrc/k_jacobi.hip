// k_jacobi.hip -- Jacobi iterations of the 2-D 9-point operator (the JacIter
// microbenchmark of Sec. 7.2.1), temporally blocked for gfx950.
//
// One iteration is x_{t+1} = (b - off * N8 x_t) / diag on an nx x ny grid
// (Dirichlet: values outside the grid are 0).  A Jacobi stencil has no
// spatial dependence, only the temporal one, so H iterations can be fused
// in LDS: a workgroup loads x and b on a (64 + 2H)^2 region around its
// 64 x 64 output tile, runs the H iterations on regions that shrink by one
// cell per side each time (the halo is recomputed by the neighbouring
// tiles, overlapped tiling), and writes the tile.  HBM traffic per pass is
// about 2 (64 + 2H)^2 + 64^2 values per 64^2 points, i.e. per iteration
// (24 + 32 H / 64 + ...) / H bytes per point instead of 24.
//
// Each thread owns one column of the region and a contiguous range of its
// rows; it walks down the rows keeping the three-value row sums of the
// previous and current row in registers, so a point costs three LDS reads,
// and takes the rows four at a time, their reads ahead of their stores.
// The two iterate buffers and b fill a CU's LDS, so one workgroup per CU:
// the launch is persistent (one workgroup per CU walking the tiles), and
// the next tile's x and b region is loaded into registers while the
// current tile iterates, so that loads and LDS work overlap.
#include "m2s_internal.hpp"

#include <algorithm>

namespace m2s {

constexpr int J9_TS = 64;    // output tile edge
constexpr int J9_NT = 1024;  // threads per workgroup: 16 wavefronts hide the
                             // LDS and load latency of the short row walks

template <int H>
__global__ void __launch_bounds__(J9_NT)
    jacobi9_tb_kernel(int nx, int ny, int tiles_x, int ntiles,
                      double inv_diag, double off,
                      const double *__restrict__ b,
                      const double *__restrict__ xin,
                      double *__restrict__ xout)
{
    constexpr int W = J9_TS + 2 * H;
    constexpr int G = J9_NT / W;  // row groups
    extern __shared__ double sm[];
    double *const xa = sm;
    double *const xb = sm + W * W;
    double *const bs = sm + 2 * W * W;
    const int tid = threadIdx.x;

    // a tile's x and b region, W^2 values each, NL per thread: loaded into
    // registers while the previous tile computes, then written to LDS
    constexpr int NL = (W * W + J9_NT - 1) / J9_NT;
    double vx[NL], vb[NL];
    auto fetch = [&](int tile) {
        const int gx0 = (tile % tiles_x) * J9_TS - H;
        const int gy0 = (tile / tiles_x) * J9_TS - H;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + q * J9_NT;
            const int ly = e / W, lx = e - (e / W) * W;
            const int gx = gx0 + lx, gy = gy0 + ly;
            const bool in =
                e < W * W && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            const long g = in ? (long)gy * nx + gx : 0;
            vx[q] = in ? xin[g] : 0.0;
            vb[q] = in ? b[g] : 0.0;
        }
    };

    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    fetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int gx0 = (tile % tiles_x) * J9_TS - H;
        const int gy0 = (tile / tiles_x) * J9_TS - H;
        __syncthreads();  // the previous tile's result has left the LDS
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + q * J9_NT;
            if (e < W * W) {
                xa[e] = vx[q];
                bs[e] = vb[q];
            }
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) fetch(tile + gridDim.x);

        const int c = tid % W, grp = tid / W;
        const int gx = gx0 + c;
        const bool colin = gx >= 0 && gx < nx;
#pragma unroll 1
        for (int t = 1; t <= H; ++t) {
            const double *src = (t & 1) ? xa : xb;
            double *dst = (t & 1) ? xb : xa;
            const int lo = t, hi = W - t;  // rows and columns computed
            // rows per group, a multiple of the 4-row groups below
            const int rows = ((hi - lo + G - 1) / G + 3) & ~3;
            const int r0 = lo + grp * rows, r1 = min(hi, r0 + rows);
            if (grp < G && c >= lo && c < hi && r0 < r1) {
                auto row3 = [&](int r, double &s3, double &side) {
                    const double *q = src + r * W + c;
                    const double l = q[-1], m = q[0], rr = q[1];
                    side = l + rr;
                    s3 = side + m;
                };
                double sp, spd, sc, scd;
                row3(r0 - 1, sp, spd);
                row3(r0, sc, scd);
                // rows in groups of four: every LDS read of a group is
                // issued before its first store (the compiler cannot tell
                // the two iterate buffers apart, so it keeps a row's reads
                // behind the previous row's store); b is read and the point
                // computed whatever `in` says, then selected, since a
                // branch around the read splits the rows into blocks too
                auto point = [&](int r, double sn, double bv) {
                    const double sum = (sp + scd) + sn;
                    const int gy = gy0 + r;
                    const bool in = colin && gy >= 0 && gy < ny;
                    const double v = (bv - off * sum) * inv_diag;
                    dst[r * W + c] = in ? v : 0.0;
                };
                int r = r0;
                for (; r + 4 <= r1; r += 4) {
                    double sn[4], snd[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        row3(r + 1 + u, sn[u], snd[u]);
                        bv[u] = bs[(r + u) * W + c];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        point(r + u, sn[u], bv[u]);
                        sp = sc;
                        sc = sn[u];
                        scd = snd[u];
                    }
                }
                for (; r < r1; ++r) {
                    double sn, snd;
                    row3(r + 1, sn, snd);
                    point(r, sn, bs[r * W + c]);
                    sp = sc;
                    sc = sn;
                    scd = snd;
                }
            }
            __syncthreads();
        }

        const double *fin = (H & 1) ? xb : xa;
        for (int e = tid; e < J9_TS * J9_TS; e += J9_NT) {
            const int ly = e / J9_TS, lx = e % J9_TS;
            const int ox = gx0 + H + lx, oy = gy0 + H + ly;
            if (ox < nx && oy < ny)
                xout[(long)oy * nx + ox] = fin[(ly + H) * W + lx + H];
        }
    }
}

template <int H>
static hipError_t jacobi9_pass(int nx, int ny, double inv_diag, double off,
                               const double *b, const double *xin,
                               double *xout, hipStream_t s)
{
    constexpr int W = J9_TS + 2 * H;
    const size_t lds = sizeof(double) * 3 * W * W;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)jacobi9_tb_kernel<H>,
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                  dev);
    if (e != hipSuccess) return e;
    const int tiles_x = (nx + J9_TS - 1) / J9_TS;
    const int ntiles = tiles_x * ((ny + J9_TS - 1) / J9_TS);
    // persistent: one workgroup per CU walks tiles blockIdx.x + k gridDim.x
    const int grid = std::max(1, std::min(ntiles, cus));
    hipLaunchKernelGGL(jacobi9_tb_kernel<H>, dim3(grid), dim3(J9_NT), lds, s,
                       nx, ny, tiles_x, ntiles, inv_diag, off, b, xin, xout);
    return hipGetLastError();
}

hipError_t launch_jacobi9(int nx, int ny, double diag, double off,
                          const double *b, double *x, double *tmp, int iters,
                          int tblock, hipStream_t s)
{
    const double inv_diag = 1.0 / diag;
    double *cur = x, *nxt = tmp;
    int left = iters;
    while (left > 0) {
        // passes of tblock iterations, the remainder in powers of two
        int h = tblock;
        while (h > left) h >>= 1;
        hipError_t e;
        switch (h) {
        case 8: e = jacobi9_pass<8>(nx, ny, inv_diag, off, b, cur, nxt, s); break;
        case 4: e = jacobi9_pass<4>(nx, ny, inv_diag, off, b, cur, nxt, s); break;
        case 2: e = jacobi9_pass<2>(nx, ny, inv_diag, off, b, cur, nxt, s); break;
        default: e = jacobi9_pass<1>(nx, ny, inv_diag, off, b, cur, nxt, s); break;
        }
        if (e != hipSuccess) return e;
        std::swap(cur, nxt);
        left -= h;
    }
    if (cur != x)
        return hipMemcpyAsync(x, cur, sizeof(double) * (size_t)nx * ny,
                              hipMemcpyDeviceToDevice, s);
    return hipSuccess;
}

}  // namespace m2s
