// k_ops.hip -- the Jacobi-style (embarrassingly parallel) stencil kernels
// around the sweeps: SpMV for the three operators (Sec. 4.3.1), the strict
// triangle parts, fused residual + injection restriction and injection
// prolongation of the multigrid cycle (the "HPCG Prolong" matrix, Table 1),
// VAR7 coarse-face construction, the face-coefficient gradient, and small
// elementwise helpers.  All are HBM-bound; loads are coalesced along x.
#include "m2s_internal.hpp"

namespace m2s {

// Deterministic block reduction of one double per thread into partials[b];
// the last block to finish sums the partials in index order into *out and
// re-arms the counter.  The partials are written and read at device scope
// (coherent across the XCDs' L2s) and each block waits for its partial's
// store before it counts itself in, so no cache-wide fence is needed.
__device__ void block_reduce_finish(double v, double *partials, double *out,
                                    unsigned *counter)
{
    __shared__ double red[1024];
    __shared__ bool last;
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y +
                                                blockDim.y * threadIdx.z);
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y +
                                              gridDim.y * blockIdx.z);
    red[tid] = v;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (s < nt && tid < s && tid + s < nt) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        __hip_atomic_store(partials + bid, red[0], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        // the partial is at the device coherence point before the count
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        unsigned prev = atomicAdd(counter, 1u);
        last = (prev == (unsigned)nb - 1);
    }
    __syncthreads();
    if (!last) return;
    double acc = 0.0;
    for (int b = tid; b < nb; b += nt)
        acc += __hip_atomic_load(partials + b, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    red[tid] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (s < nt && tid < s && tid + s < nt) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        *out = red[0];
        *counter = 0u;
    }
}

// --------------------------------------------------------------------------
// CONST27 SpMV.  A workgroup owns a 64 x 16 (x, y) tile of one layer of kc
// planes and marches through the layer plane by plane.  Each plane of the
// tile plus its 1-point halo is staged in LDS; its loads are issued two
// planes ahead into registers, so two planes per workgroup are in flight
// while the current one is summed.  A thread owns one x column of 4
// consecutive rows (8 in FP32, whose tiles are 64 x 32: the same bytes per
// staged plane) and keeps their 3x3 plane sums of the planes on either side
// in registers; the 3x3 sums are built from row sums (3 LDS reads per row,
// 6 rows for 4 points), so every x value is read from HBM once per layer,
// and the halo rows and columns come from L2 when the tile that owns them
// runs at the same time.
//
// Placement: workgroup w runs on XCD w mod 8, so the tiles (numbered layer
// by layer, x fastest) are handed to the XCDs in contiguous blocks: the
// tiles running together on one XCD are spatial neighbours and share their
// halos in that XCD's L2.  About 512 workgroups (two per CU, 8 waves):
// fewer leave too few loads in flight, more cut the layers thinner.
//   y = diag * x + off * ((S9(k-1) + S8(k)) + S9(k+1))
// S9 = 3x3 sum in a plane, S8 = the same without the centre.
// --------------------------------------------------------------------------
constexpr int SP_TX = 64, SP_W = SP_TX + 2;
constexpr int SP_TARGET_WGS = 512;

template <typename T>
struct SpCfg {
    static constexpr int TY = sizeof(T) == 8 ? 16 : 32;
    static constexpr int R = TY / 4;  // rows per thread
    static constexpr int H = TY + 2;
    static constexpr int NQ = (SP_W * H + 255) / 256;  // staged values/thread
};

struct SpTiles {
    int nbx, nby, kc, ntiles, per_xcd;
};

SpTiles sp_tiles(const Grid &g, int ty)
{
    SpTiles t;
    t.nbx = (g.nx + SP_TX - 1) / SP_TX;
    t.nby = (g.ny + ty - 1) / ty;
    const int tpl = t.nbx * t.nby;
    int layers = std::max(1, std::min(g.nz, (SP_TARGET_WGS + tpl - 1) / tpl));
    t.kc = (g.nz + layers - 1) / layers;
    layers = (g.nz + t.kc - 1) / t.kc;
    t.ntiles = layers * tpl;
    t.per_xcd = (t.ntiles + 7) / 8;
    return t;
}

template <typename T, bool DOT>
__global__ void __launch_bounds__(256)
    spmv27_kernel(Grid g, SpTiles t, T diag, T off, const T *__restrict__ x,
                  T *__restrict__ y, double *partials, double *dot_out,
                  unsigned *counter)
{
    constexpr int SP_TY = SpCfg<T>::TY, SP_R = SpCfg<T>::R;
    constexpr int SP_H = SpCfg<T>::H, SP_NQ = SpCfg<T>::NQ;
    __shared__ T pl[2][SP_H][SP_W];
    const int tid = threadIdx.x;
    const int id = (int)(blockIdx.x % 8) * t.per_xcd + (int)(blockIdx.x / 8);
    double acc = 0.0;
    if (id < t.ntiles) {
        const int tpl = t.nbx * t.nby;
        const int layer = id / tpl, tile = id - layer * tpl;
        const int i0 = (tile % t.nbx) * SP_TX, j0 = (tile / t.nbx) * SP_TY;
        const int ka = layer * t.kc, kb = min(g.nz, ka + t.kc);
        const int n = kb - ka;
        const int64_t plane = (int64_t)g.nx * g.ny;

        // staging slots of this thread: offset within a plane, -1 outside
        // the grid (staged as 0), -2 no slot
        int goff[SP_NQ];
#pragma unroll
        for (int q = 0; q < SP_NQ; ++q) {
            const int e = tid + 256 * q;
            goff[q] = -2;
            if (e < SP_W * SP_H) {
                const int row = e / SP_W, col = e - (e / SP_W) * SP_W;
                const int i = i0 - 1 + col, j = j0 - 1 + row;
                goff[q] = (i >= 0 && i < g.nx && j >= 0 && j < g.ny)
                              ? j * g.nx + i
                              : -1;
            }
        }
        auto load = [&](T(&r)[SP_NQ], int k) {
            const bool kin = k >= 0 && k < g.nz;
            const T *xk = x + (int64_t)k * plane;
#pragma unroll
            for (int q = 0; q < SP_NQ; ++q)
                r[q] = (kin && goff[q] >= 0) ? xk[goff[q]] : T(0);
        };
        auto store = [&](int b, const T(&r)[SP_NQ]) {
            T *flat = &pl[b][0][0];
#pragma unroll
            for (int q = 0; q < SP_NQ; ++q)
                if (goff[q] != -2) flat[tid + 256 * q] = r[q];
        };
        const int tx = tid & 63, ty = tid >> 6;
        // 3x3 sums of the thread's SP_R rows in the plane staged in buffer b
        auto sums = [&](int b, T(&s9)[SP_R], T(&s8)[SP_R], T(&c)[SP_R]) {
            T rs[SP_R + 2], bb[SP_R];
#pragma unroll
            for (int rr = 0; rr < SP_R + 2; ++rr) {
                const T *row = &pl[b][ty * SP_R + rr][tx];
                const T xl = row[0], xc = row[1], xr = row[2];
                rs[rr] = (xl + xc) + xr;
                if (rr >= 1 && rr <= SP_R) {
                    bb[rr - 1] = xl + xr;
                    c[rr - 1] = xc;
                }
            }
#pragma unroll
            for (int r = 0; r < SP_R; ++r) {
                s8[r] = (rs[r] + bb[r]) + rs[r + 2];
                s9[r] = (rs[r] + (bb[r] + c[r])) + rs[r + 2];
            }
        };
        const int i = i0 + tx;
        // sums of the plane behind (p) and the current plane (s9c, s8c, cc)
        T s9p[SP_R], s9c[SP_R], s8c[SP_R], cc[SP_R], d8[SP_R], dc[SP_R];
        T ra[SP_NQ], rb[SP_NQ];
        load(ra, ka - 1);
        load(rb, ka);
        store(0, ra);
        load(ra, ka + 1);
        __syncthreads();
        sums(0, s9p, d8, dc);
        store(1, rb);
        if (n >= 2) load(rb, ka + 2);
        __syncthreads();
        sums(1, s9c, s8c, cc);
        // one plane: stage plane k + 1 from r, prefetch k + 3 into r, sum
        // the staged plane and write y at plane k
        auto step = [&](T(&r)[SP_NQ], int s, int b) {
            const int k = ka + s;
            store(b, r);
            if (s + 3 <= n) load(r, k + 3);
            __syncthreads();
            T s9n[SP_R], s8n[SP_R], cn[SP_R];
            sums(b, s9n, s8n, cn);
            T *yk = y + (int64_t)k * plane;
#pragma unroll
            for (int rr = 0; rr < SP_R; ++rr) {
                const int j = j0 + ty * SP_R + rr;
                if (i < g.nx && j < g.ny) {
                    const T nb = (s9p[rr] + s8c[rr]) + s9n[rr];
                    const T v = fma(off, nb, diag * cc[rr]);
                    yk[j * g.nx + i] = v;
                    if (DOT) acc = fma((double)cc[rr], (double)v, acc);
                }
                s9p[rr] = s9c[rr];
                s9c[rr] = s9n[rr];
                s8c[rr] = s8n[rr];
                cc[rr] = cn[rr];
            }
        };
        for (int s = 0; s < n; s += 2) {
            step(ra, s, 0);
            if (s + 1 < n) step(rb, s + 1, 1);
        }
    }
    if (DOT) block_reduce_finish(acc, partials, dot_out, counter);
}

// The grid-stride loops of the reduction kernels load RED_U strides ahead
// before they accumulate, in the same order as the plain loop, so that each
// thread has several loads in flight (one at a time leaves them
// latency-bound).
constexpr int RED_U = 4;

// --------------------------------------------------------------------------
// VAR7 SpMV (optionally fused with x.y).
// --------------------------------------------------------------------------
template <typename T, bool DOT>
__global__ void __launch_bounds__(256)
    spmv_var7_kernel(Grid g, const T *__restrict__ kx,
                     const T *__restrict__ ky, const T *__restrict__ kz,
                     const T *__restrict__ x, T *__restrict__ y,
                     double *partials, double *dot_out, unsigned *counter)
{
    Faces F{g.nx, g.ny, g.nz};
    double acc = 0.0;
    const int64_t n = g.size();
    const int64_t pl = (int64_t)g.nx * g.ny;
    auto point = [&](int64_t p, T &xc, T &v) {
        const int i = (int)(p % g.nx);
        const int64_t t = p / g.nx;
        const int j = (int)(t % g.ny), k = (int)(t / g.ny);
        const T kxm = kx[F.ix(i, j, k)], kxp = kx[F.ix(i + 1, j, k)];
        const T kym = ky[F.iy(i, j, k)], kyp = ky[F.iy(i, j + 1, k)];
        const T kzm = kz[F.iz(i, j, k)], kzp = kz[F.iz(i, j, k + 1)];
        xc = x[p];
        const T vmx = i > 0 ? x[p - 1] : T(0);
        const T vpx = i < g.nx - 1 ? x[p + 1] : T(0);
        const T vmy = j > 0 ? x[p - g.nx] : T(0);
        const T vpy = j < g.ny - 1 ? x[p + g.nx] : T(0);
        const T vmz = k > 0 ? x[p - pl] : T(0);
        const T vpz = k < g.nz - 1 ? x[p + pl] : T(0);
        T d = ((kxm + kxp) + (kym + kyp)) + (kzm + kzp);
        T s1 = fma(kxm, vmx, kxp * vpx);
        T s2 = fma(kym, vmy, kyp * vpy);
        T s3 = fma(kzm, vmz, kzp * vpz);
        v = fma(d, xc, -((s1 + s2) + s3));
    };
    // RED_U points per trip, their loads ahead of the stores and of the
    // accumulation (which keeps the plain loop's order)
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; p + (RED_U - 1) * st < n; p += RED_U * st) {
        T xc[RED_U], v[RED_U];
#pragma unroll
        for (int u = 0; u < RED_U; ++u) point(p + u * st, xc[u], v[u]);
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            y[p + u * st] = v[u];
            if (DOT) acc = fma((double)xc[u], (double)v[u], acc);
        }
    }
    for (; p < n; p += st) {
        T xc, v;
        point(p, xc, v);
        y[p] = v;
        if (DOT) acc = fma((double)xc, (double)v, acc);
    }
    if (DOT) block_reduce_finish(acc, partials, dot_out, counter);
}

// --------------------------------------------------------------------------
// BLOCK7 SpMV.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    spmv_block7_kernel(Grid g, Block7Consts C, const double *__restrict__ x,
                       double *__restrict__ y)
{
    const int64_t n = g.size();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % g.nx);
        const int64_t t = p / g.nx;
        const int j = (int)(t % g.ny), k = (int)(t / g.ny);
        const int di[7] = {0, -1, 1, 0, 0, 0, 0};
        const int dj[7] = {0, 0, 0, -1, 1, 0, 0};
        const int dk[7] = {0, 0, 0, 0, 0, -1, 1};
        double s[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            const int ii = i + di[d], jj = j + dj[d], kk = k + dk[d];
            if (!g.in(ii, jj, kk)) continue;
            const int64_t q = 5 * g.idx(ii, jj, kk);
            double xq[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) xq[c] = x[q + c];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    s[a] = fma(C.B[d][5 * a + c], xq[c], s[a]);
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) y[5 * p + a] = s[a];
    }
}

// --------------------------------------------------------------------------
// Strict lower / upper triangle parts (CONST27, VAR7).
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
    spmv_part_kernel(Grid g, int kind, int part, T off, const T *kx,
                     const T *ky, const T *kz, const T *__restrict__ x,
                     T *__restrict__ y)
{
    Faces F{g.nx, g.ny, g.nz};
    const int64_t n = g.size();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % g.nx);
        const int64_t t = p / g.nx;
        const int j = (int)(t % g.ny), k = (int)(t / g.ny);
        T s = T(0);
        if (kind == M2S_CONST27) {
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int o = (dz * 3 + dy) * 3 + dx;
                        if (o == 0 || (part < 0) != (o < 0)) continue;
                        if (!g.in(i + dx, j + dy, k + dz)) continue;
                        s += x[g.idx(i + dx, j + dy, k + dz)];
                    }
            s = off * s;
        } else {
            if (part < 0) {
                T a = k > 0 ? kz[F.iz(i, j, k)] * x[g.idx(i, j, k - 1)] : T(0);
                T b = j > 0 ? ky[F.iy(i, j, k)] * x[g.idx(i, j - 1, k)] : T(0);
                T c = i > 0 ? kx[F.ix(i, j, k)] * x[g.idx(i - 1, j, k)] : T(0);
                s = -((a + b) + c);
            } else {
                T a = i < g.nx - 1 ? kx[F.ix(i + 1, j, k)] *
                                         x[g.idx(i + 1, j, k)]
                                   : T(0);
                T b = j < g.ny - 1 ? ky[F.iy(i, j + 1, k)] *
                                         x[g.idx(i, j + 1, k)]
                                   : T(0);
                T c = k < g.nz - 1 ? kz[F.iz(i, j, k + 1)] *
                                         x[g.idx(i, j, k + 1)]
                                   : T(0);
                s = -((a + b) + c);
            }
        }
        y[p] = s;
    }
}

// --------------------------------------------------------------------------
// Fused residual + injection restriction: rc[I,J,K] = r - A z at the fine
// point (2I, 2J, 2K).
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
    restrict_kernel(Grid gf, int kind, T diag, T off, const T *kx,
                    const T *ky, const T *kz, const T *__restrict__ r,
                    const T *__restrict__ z, T *__restrict__ rc)
{
    const Grid gc{gf.nx / 2, gf.ny / 2, gf.nz / 2};
    Faces F{gf.nx, gf.ny, gf.nz};
    const int64_t n = gc.size();
    for (int64_t pc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < n;
         pc += (int64_t)gridDim.x * blockDim.x) {
        const int I = (int)(pc % gc.nx);
        const int64_t t = pc / gc.nx;
        const int J = (int)(t % gc.ny), K = (int)(t / gc.ny);
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        const int64_t p = gf.idx(i, j, k);
        T az;
        if (kind == M2S_CONST27) {
            T s = T(0);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy) {
                    T row = T(0);
                    for (int dx = -1; dx <= 1; ++dx) {
                        if ((dx | dy | dz) == 0) continue;
                        if (!gf.in(i + dx, j + dy, k + dz)) continue;
                        row += z[gf.idx(i + dx, j + dy, k + dz)];
                    }
                    s += row;
                }
            az = fma(off, s, diag * z[p]);
        } else {
            const T kxm = kx[F.ix(i, j, k)], kxp = kx[F.ix(i + 1, j, k)];
            const T kym = ky[F.iy(i, j, k)], kyp = ky[F.iy(i, j + 1, k)];
            const T kzm = kz[F.iz(i, j, k)], kzp = kz[F.iz(i, j, k + 1)];
            const T vmx = i > 0 ? z[p - 1] : T(0);
            const T vpx = i < gf.nx - 1 ? z[p + 1] : T(0);
            const T vmy = j > 0 ? z[p - gf.nx] : T(0);
            const T vpy = j < gf.ny - 1 ? z[p + gf.nx] : T(0);
            const int64_t pl = (int64_t)gf.nx * gf.ny;
            const T vmz = k > 0 ? z[p - pl] : T(0);
            const T vpz = k < gf.nz - 1 ? z[p + pl] : T(0);
            T d = ((kxm + kxp) + (kym + kyp)) + (kzm + kzp);
            T s1 = fma(kxm, vmx, kxp * vpx);
            T s2 = fma(kym, vmy, kyp * vpy);
            T s3 = fma(kzm, vmz, kzp * vpz);
            az = fma(d, z[p], -((s1 + s2) + s3));
        }
        rc[pc] = r[p] - az;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
    prolong_kernel(Grid gf, const T *__restrict__ zc, T *__restrict__ z)
{
    const Grid gc{gf.nx / 2, gf.ny / 2, gf.nz / 2};
    const int64_t n = gc.size();
    for (int64_t pc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pc < n;
         pc += (int64_t)gridDim.x * blockDim.x) {
        const int I = (int)(pc % gc.nx);
        const int64_t t = pc / gc.nx;
        const int J = (int)(t % gc.ny), K = (int)(t / gc.ny);
        const int64_t p = gf.idx(2 * I, 2 * J, 2 * K);
        z[p] += zc[pc];
    }
}

// Coarse VAR7 faces: half the conductance of the fine segment a coarse face
// spans, eliminated exactly on a 1-D line.  Interior and last faces span two
// fine faces in series: ab / (2 (a + b)); the first face on an axis spans
// fine face 0 only (coarse point 0 is fine point 0): k0 / 2.  Transverse
// position on the coincident fine row.
template <typename T>
__device__ __forceinline__ T half_series(T a, T b)
{
    return (a * b) / (T(2) * (a + b));
}

template <typename T>
__global__ void __launch_bounds__(256)
    coarsen_kernel(Grid gf, const T *kx, const T *ky, const T *kz, T *kxc,
                   T *kyc, T *kzc)
{
    const Grid gc{gf.nx / 2, gf.ny / 2, gf.nz / 2};
    Faces Ff{gf.nx, gf.ny, gf.nz}, Fc{gc.nx, gc.ny, gc.nz};
    const int64_t nx = Fc.nfx(), ny = Fc.nfy(), nz = Fc.nfz();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         e < nx + ny + nz; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nx) {
            const int I = (int)(e % (gc.nx + 1));
            const int64_t t = e / (gc.nx + 1);
            const int J = (int)(t % gc.ny), K = (int)(t / gc.ny);
            kxc[e] = I == 0 ? kx[Ff.ix(0, 2 * J, 2 * K)] / T(2)
                            : half_series(kx[Ff.ix(2 * I - 1, 2 * J, 2 * K)],
                                          kx[Ff.ix(2 * I, 2 * J, 2 * K)]);
        } else if (e < nx + ny) {
            const int64_t f = e - nx;
            const int I = (int)(f % gc.nx);
            const int64_t t = f / gc.nx;
            const int J = (int)(t % (gc.ny + 1)), K = (int)(t / (gc.ny + 1));
            kyc[f] = J == 0 ? ky[Ff.iy(2 * I, 0, 2 * K)] / T(2)
                            : half_series(ky[Ff.iy(2 * I, 2 * J - 1, 2 * K)],
                                          ky[Ff.iy(2 * I, 2 * J, 2 * K)]);
        } else {
            const int64_t f = e - nx - ny;
            const int I = (int)(f % gc.nx);
            const int64_t t = f / gc.nx;
            const int J = (int)(t % gc.ny), K = (int)(t / gc.ny);
            kzc[f] = K == 0 ? kz[Ff.iz(2 * I, 2 * J, 0)] / T(2)
                            : half_series(kz[Ff.iz(2 * I, 2 * J, 2 * K - 1)],
                                          kz[Ff.iz(2 * I, 2 * J, 2 * K)]);
        }
    }
}

// dL/dk_f = -(lam_p - lam_q)(u_p - u_q), zero ghosts.
__global__ void __launch_bounds__(256)
    face_grad_kernel(Grid g, const double *__restrict__ u,
                     const double *__restrict__ lam, double *gx, double *gy,
                     double *gz)
{
    Faces F{g.nx, g.ny, g.nz};
    const int64_t nfx = F.nfx(), nfy = F.nfy(), nfz = F.nfz();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         e < nfx + nfy + nfz; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k, dx = 0, dy = 0, dz = 0;
        double *out;
        int64_t f;
        if (e < nfx) {
            f = e;
            i = (int)(f % (g.nx + 1));
            const int64_t t = f / (g.nx + 1);
            j = (int)(t % g.ny);
            k = (int)(t / g.ny);
            dx = 1;
            out = gx;
        } else if (e < nfx + nfy) {
            f = e - nfx;
            i = (int)(f % g.nx);
            const int64_t t = f / g.nx;
            j = (int)(t % (g.ny + 1));
            k = (int)(t / (g.ny + 1));
            dy = 1;
            out = gy;
        } else {
            f = e - nfx - nfy;
            i = (int)(f % g.nx);
            const int64_t t = f / g.nx;
            j = (int)(t % g.ny);
            k = (int)(t / g.ny);
            dz = 1;
            out = gz;
        }
        // face between a = (i,j,k) - d and b = (i,j,k)
        const int ia = i - dx, ja = j - dy, ka = k - dz;
        const bool ina = g.in(ia, ja, ka), inb = g.in(i, j, k);
        const double ua = ina ? u[g.idx(ia, ja, ka)] : 0.0;
        const double la = ina ? lam[g.idx(ia, ja, ka)] : 0.0;
        const double ub = inb ? u[g.idx(i, j, k)] : 0.0;
        const double lb = inb ? lam[g.idx(i, j, k)] : 0.0;
        out[f] = -(lb - la) * (ub - ua);
    }
}

template <typename S, typename D>
__global__ void __launch_bounds__(256)
    convert_kernel(const S *__restrict__ s, D *__restrict__ d, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        d[p] = (D)s[p];
}

template <typename T>
__global__ void __launch_bounds__(256) fill_kernel(T *d, int64_t n, T v)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        d[p] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) scale_kernel(T *d, int64_t n, T a)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        d[p] *= a;
}

template <typename T>
__global__ void __launch_bounds__(256)
    add_kernel(T *__restrict__ d, const T *__restrict__ s, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        d[p] += s[p];
}

__global__ void __launch_bounds__(256)
    copy_kernel(const double4 *__restrict__ s, double4 *__restrict__ d,
                int64_t n4, const char *__restrict__ stail,
                char *__restrict__ dtail, int tail)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n4;
         p += (int64_t)gridDim.x * blockDim.x)
        d[p] = s[p];
    if (blockIdx.x == 0 && (int)threadIdx.x < tail)
        dtail[threadIdx.x] = stail[threadIdx.x];
}

// --------------------------------------------------------------------------
// CG vector kernels (double) with deterministic reductions.
// --------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
int dot_partials_capacity() { return kRedBlocks + 8; }

// partials layout: [0, kRedBlocks) per-block values, then a counter word.
static unsigned *counter_of(double *partials)
{
    return (unsigned *)(partials + kRedBlocks);
}

__global__ void __launch_bounds__(256)
    dot_kernel(const double *__restrict__ x, const double *__restrict__ y,
               int64_t n, double *partials, double *out, unsigned *counter)
{
    double acc = 0.0;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; p + (RED_U - 1) * st < n; p += RED_U * st) {
        double xv[RED_U], yv[RED_U];
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            xv[u] = x[p + u * st];
            yv[u] = y[p + u * st];
        }
#pragma unroll
        for (int u = 0; u < RED_U; ++u) acc = fma(xv[u], yv[u], acc);
    }
    for (; p < n; p += st) acc = fma(x[p], y[p], acc);
    block_reduce_finish(acc, partials, out, counter);
}

__global__ void __launch_bounds__(256)
    residual_kernel(const double *__restrict__ b, const double *__restrict__ ax,
                    double *__restrict__ r, int64_t n, double *partials,
                    double *out, unsigned *counter)
{
    double acc = 0.0;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; p + (RED_U - 1) * st < n; p += RED_U * st) {
        double bv[RED_U], av[RED_U];
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            bv[u] = b[p + u * st];
            av[u] = ax[p + u * st];
        }
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            const double v = bv[u] - av[u];
            r[p + u * st] = v;
            acc = fma(v, v, acc);
        }
    }
    for (; p < n; p += st) {
        const double v = b[p] - ax[p];
        r[p] = v;
        acc = fma(v, v, acc);
    }
    block_reduce_finish(acc, partials, out, counter);
}

__global__ void __launch_bounds__(256)
    update_p_kernel(const double *__restrict__ z, double *__restrict__ p,
                    int64_t n, const double *sc, int first)
{
    // SC_BD is written only by update_xr of an earlier iteration
    if (sc[SC_BD] != 0.0) return;
    const double beta = first ? 0.0 : sc[SC_RZ] / sc[SC_RZ_OLD];
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = first ? z[q] : fma(beta, p[q], z[q]);
}

__global__ void __launch_bounds__(256)
    update_xr_kernel(double *__restrict__ x, double *__restrict__ r,
                     const double *__restrict__ p,
                     const double *__restrict__ ap, int64_t n, double *sc,
                     double *partials, unsigned *counter, int iter)
{
    const double rz = sc[SC_RZ], pap = sc[SC_PAP];
    const double alpha = rz / pap;
    // every block computes `bad` from the same scalars; one latches it.  A
    // block that already sees this launch's latch skips as well, since it
    // then has bad set too
    const bool bad = !(pap > 0.0) || !isfinite(pap) || !isfinite(rz);
    const bool skip = bad || sc[SC_BD] != 0.0;
    if (bad && blockIdx.x == 0 && threadIdx.x == 0 && sc[SC_BD] == 0.0) {
        sc[SC_BDIT] = (double)iter;
        sc[SC_BD] = 1.0;
    }
    double acc = 0.0;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (skip) q = n;
    for (; q + (RED_U - 1) * st < n; q += RED_U * st) {
        double xv[RED_U], pv[RED_U], rv[RED_U], av[RED_U];
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            xv[u] = x[q + u * st];
            pv[u] = p[q + u * st];
            rv[u] = r[q + u * st];
            av[u] = ap[q + u * st];
        }
#pragma unroll
        for (int u = 0; u < RED_U; ++u) {
            x[q + u * st] = fma(alpha, pv[u], xv[u]);
            const double v = fma(-alpha, av[u], rv[u]);
            r[q + u * st] = v;
            acc = fma(v, v, acc);
        }
    }
    for (; q < n; q += st) {
        x[q] = fma(alpha, p[q], x[q]);
        const double v = fma(-alpha, ap[q], r[q]);
        r[q] = v;
        acc = fma(v, v, acc);
    }
    block_reduce_finish(acc, partials, sc + SC_RR, counter);
}

static int blocks_for(int64_t n, int threads = 256, int cap = 8192)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// --------------------------------------------------------------------------
// Host launchers.
// --------------------------------------------------------------------------
template <typename T, bool DOT>
static hipError_t sp27(const m2s_stencil &A, const void *x, void *y,
                       double *partials, double *out, hipStream_t s)
{
    Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const SpTiles t = sp_tiles(g, SpCfg<T>::TY);
    const dim3 block(256), grid(8 * t.per_xcd);
    if (DOT && (int64_t)grid.x > kRedBlocks) {
        // too many blocks for the partials buffer: plain SpMV then a dot
        hipLaunchKernelGGL((spmv27_kernel<T, false>), grid, block, 0, s, g, t,
                           (T)A.diag, (T)A.offdiag, (const T *)x, (T *)y,
                           nullptr, nullptr, nullptr);
        hipLaunchKernelGGL(dot_kernel, dim3(blocks_for(g.size(), 256,
                                                       kRedBlocks)),
                           dim3(256), 0, s, (const double *)x,
                           (const double *)y, g.size(), partials, out,
                           counter_of(partials));
        return hipGetLastError();
    }
    hipLaunchKernelGGL((spmv27_kernel<T, DOT>), grid, block, 0, s, g, t,
                       (T)A.diag, (T)A.offdiag, (const T *)x, (T *)y,
                       partials, out, DOT ? counter_of(partials) : nullptr);
    return hipGetLastError();
}

template <typename T, bool DOT>
static hipError_t spv7(const m2s_stencil &A, const void *x, void *y,
                       double *partials, double *out, hipStream_t s)
{
    Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int nb = blocks_for(g.size(), 256, DOT ? kRedBlocks : 8192);
    hipLaunchKernelGGL((spmv_var7_kernel<T, DOT>), dim3(nb), dim3(256), 0, s,
                       g, (const T *)A.kx, (const T *)A.ky, (const T *)A.kz,
                       (const T *)x, (T *)y, partials, out,
                       DOT ? counter_of(partials) : nullptr);
    return hipGetLastError();
}

hipError_t fill_block7_consts(const double *blocks_host, Block7Consts &C);

hipError_t launch_spmv(const m2s_stencil &A, const void *x, void *y,
                       hipStream_t s)
{
    switch (A.kind) {
    case M2S_CONST27:
        return A.dtype == M2S_F64
                   ? sp27<double, false>(A, x, y, nullptr, nullptr, s)
                   : sp27<float, false>(A, x, y, nullptr, nullptr, s);
    case M2S_VAR7:
        return A.dtype == M2S_F64
                   ? spv7<double, false>(A, x, y, nullptr, nullptr, s)
                   : spv7<float, false>(A, x, y, nullptr, nullptr, s);
    case M2S_BLOCK7_5: {
        Block7Consts C{};
        hipError_t e = fill_block7_consts(A.blocks, C);
        if (e != hipSuccess) return e;
        Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
        hipLaunchKernelGGL(spmv_block7_kernel, dim3(blocks_for(g.size())),
                           dim3(256), 0, s, g, C, (const double *)x,
                           (double *)y);
        return hipGetLastError();
    }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_spmv_dot(const m2s_stencil &A, const double *p, double *ap,
                           double *partials, double *out, hipStream_t s)
{
    if (A.kind == M2S_CONST27) return sp27<double, true>(A, p, ap, partials, out, s);
    return spv7<double, true>(A, p, ap, partials, out, s);
}

hipError_t launch_spmv_part(const m2s_stencil &A, int part, const void *x,
                            void *y, hipStream_t s)
{
    Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int nb = blocks_for(g.size());
    if (A.dtype == M2S_F64)
        hipLaunchKernelGGL(spmv_part_kernel<double>, dim3(nb), dim3(256), 0,
                           s, g, (int)A.kind, part, A.offdiag,
                           (const double *)A.kx, (const double *)A.ky,
                           (const double *)A.kz, (const double *)x,
                           (double *)y);
    else
        hipLaunchKernelGGL(spmv_part_kernel<float>, dim3(nb), dim3(256), 0, s,
                           g, (int)A.kind, part, (float)A.offdiag,
                           (const float *)A.kx, (const float *)A.ky,
                           (const float *)A.kz, (const float *)x,
                           (float *)y);
    return hipGetLastError();
}

hipError_t launch_restrict(const m2s_stencil &A, const void *r, const void *z,
                           void *rc, hipStream_t s)
{
    Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int nb = blocks_for(g.size() / 8 + 1);
    if (A.dtype == M2S_F64)
        hipLaunchKernelGGL(restrict_kernel<double>, dim3(nb), dim3(256), 0, s,
                           g, (int)A.kind, A.diag, A.offdiag,
                           (const double *)A.kx, (const double *)A.ky,
                           (const double *)A.kz, (const double *)r,
                           (const double *)z, (double *)rc);
    else
        hipLaunchKernelGGL(restrict_kernel<float>, dim3(nb), dim3(256), 0, s,
                           g, (int)A.kind, (float)A.diag, (float)A.offdiag,
                           (const float *)A.kx, (const float *)A.ky,
                           (const float *)A.kz, (const float *)r,
                           (const float *)z, (float *)rc);
    return hipGetLastError();
}

hipError_t launch_prolong(const m2s_stencil &A, const void *zc, void *z,
                          hipStream_t s)
{
    Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int nb = blocks_for(g.size() / 8 + 1);
    if (A.dtype == M2S_F64)
        hipLaunchKernelGGL(prolong_kernel<double>, dim3(nb), dim3(256), 0, s,
                           g, (const double *)zc, (double *)z);
    else
        hipLaunchKernelGGL(prolong_kernel<float>, dim3(nb), dim3(256), 0, s,
                           g, (const float *)zc, (float *)z);
    return hipGetLastError();
}

hipError_t launch_var7_coarsen(m2s_dtype t, Grid fine, const void *kx,
                               const void *ky, const void *kz, void *kxc,
                               void *kyc, void *kzc, hipStream_t s)
{
    const int nb = blocks_for(fine.size() / 2 + 64);
    if (t == M2S_F64)
        hipLaunchKernelGGL(coarsen_kernel<double>, dim3(nb), dim3(256), 0, s,
                           fine, (const double *)kx, (const double *)ky,
                           (const double *)kz, (double *)kxc, (double *)kyc,
                           (double *)kzc);
    else
        hipLaunchKernelGGL(coarsen_kernel<float>, dim3(nb), dim3(256), 0, s,
                           fine, (const float *)kx, (const float *)ky,
                           (const float *)kz, (float *)kxc, (float *)kyc,
                           (float *)kzc);
    return hipGetLastError();
}

hipError_t launch_face_grad(Grid g, const double *u, const double *lam,
                            double *gx, double *gy, double *gz, hipStream_t s)
{
    Faces F{g.nx, g.ny, g.nz};
    const int nb = blocks_for(F.nfx() + F.nfy() + F.nfz());
    hipLaunchKernelGGL(face_grad_kernel, dim3(nb), dim3(256), 0, s, g, u, lam,
                       gx, gy, gz);
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, m2s_dtype st, void *dst,
                          m2s_dtype dt, int64_t n, hipStream_t s)
{
    const int nb = blocks_for(n);
    if (st == M2S_F64 && dt == M2S_F32)
        hipLaunchKernelGGL((convert_kernel<double, float>), dim3(nb),
                           dim3(256), 0, s, (const double *)src, (float *)dst,
                           n);
    else if (st == M2S_F32 && dt == M2S_F64)
        hipLaunchKernelGGL((convert_kernel<float, double>), dim3(nb),
                           dim3(256), 0, s, (const float *)src,
                           (double *)dst, n);
    else if (st == M2S_F64)
        hipLaunchKernelGGL((convert_kernel<double, double>), dim3(nb),
                           dim3(256), 0, s, (const double *)src,
                           (double *)dst, n);
    else
        hipLaunchKernelGGL((convert_kernel<float, float>), dim3(nb),
                           dim3(256), 0, s, (const float *)src, (float *)dst,
                           n);
    return hipGetLastError();
}

hipError_t launch_fill(void *dst, m2s_dtype t, int64_t n, double v,
                       hipStream_t s)
{
    const int nb = blocks_for(n);
    if (t == M2S_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(nb), dim3(256), 0, s,
                           (double *)dst, n, v);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(nb), dim3(256), 0, s,
                           (float *)dst, n, (float)v);
    return hipGetLastError();
}

hipError_t launch_scale(void *x, m2s_dtype t, int64_t n, double a,
                        hipStream_t s)
{
    const int nb = blocks_for(n);
    if (t == M2S_F64)
        hipLaunchKernelGGL(scale_kernel<double>, dim3(nb), dim3(256), 0, s,
                           (double *)x, n, a);
    else
        hipLaunchKernelGGL(scale_kernel<float>, dim3(nb), dim3(256), 0, s,
                           (float *)x, n, (float)a);
    return hipGetLastError();
}

hipError_t launch_add(void *x, const void *y, m2s_dtype t, int64_t n,
                      hipStream_t s)
{
    const int nb = blocks_for(n);
    if (t == M2S_F64)
        hipLaunchKernelGGL(add_kernel<double>, dim3(nb), dim3(256), 0, s,
                           (double *)x, (const double *)y, n);
    else
        hipLaunchKernelGGL(add_kernel<float>, dim3(nb), dim3(256), 0, s,
                           (float *)x, (const float *)y, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, int64_t bytes,
                       hipStream_t s)
{
    if (((uintptr_t)dst | (uintptr_t)src) & 31)
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
    const int64_t n4 = bytes / 32;
    const int tail = (int)(bytes - n4 * 32);
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(n4 + 1)), dim3(256), 0, s,
                       (const double4 *)src, (double4 *)dst, n4,
                       (const char *)src + n4 * 32, (char *)dst + n4 * 32,
                       tail);
    return hipGetLastError();
}

// STREAM-style reference kernels (the measured HBM rate of a plain
// streaming pass, beside the nominal peak): copy c = a, triad c = a + s b.
// One 16-byte pair of doubles per thread, one wave of workgroups over the
// whole array (measured on MI355X against 2, 4 and 8 pairs per thread and
// non-temporal accesses: this plain form is the fastest, 6.2 / 6.0 TB/s
// over 1 GiB arrays); thread 0 also takes an odd last element.
template <int KIND>
__global__ void __launch_bounds__(256)
    stream_kernel(const double *__restrict__ a, const double *__restrict__ b,
                  double *__restrict__ c, double sc, int64_t n)
{
    using d2 = __attribute__((ext_vector_type(2))) double;
    const int64_t n2 = n / 2;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n2) {
        const d2 x = ((const d2 *)a)[q];
        if constexpr (KIND == 0) ((d2 *)c)[q] = x;
        else ((d2 *)c)[q] = x + sc * ((const d2 *)b)[q];
    }
    if (q == 0 && (n & 1)) {
        if constexpr (KIND == 0) c[n - 1] = a[n - 1];
        else c[n - 1] = a[n - 1] + sc * b[n - 1];
    }
}

hipError_t launch_stream(int kind, const double *a, const double *b,
                         double *c, double sc, int64_t n, hipStream_t s)
{
    const int64_t nb = std::max<int64_t>(1, (n / 2 + 255) / 256);
    if (nb >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    if (kind == 0)
        hipLaunchKernelGGL(stream_kernel<0>, dim3((unsigned)nb), dim3(256), 0,
                           s, a, b, c, sc, n);
    else
        hipLaunchKernelGGL(stream_kernel<1>, dim3((unsigned)nb), dim3(256), 0,
                           s, a, b, c, sc, n);
    return hipGetLastError();
}

// Zero the counter word of a partials buffer (a kernel, not a memset, so
// that the call can sit in a captured graph).
hipError_t launch_dot_reset(double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel<double>, dim3(1), dim3(256), 0, s,
                       partials + kRedBlocks, (int64_t)1, 0.0);
    return hipGetLastError();
}

hipError_t launch_dot(const double *x, const double *y, int64_t n,
                      double *partials, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(dot_kernel, dim3(blocks_for(n, 256, kRedBlocks)),
                       dim3(256), 0, s, x, y, n, partials, out,
                       counter_of(partials));
    return hipGetLastError();
}

hipError_t launch_residual(const double *b, const double *ax, double *r,
                           int64_t n, double *partials, double *rr_out,
                           hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(blocks_for(n, 256, kRedBlocks)),
                       dim3(256), 0, s, b, ax, r, n, partials, rr_out,
                       counter_of(partials));
    return hipGetLastError();
}

hipError_t launch_update_p(const double *z, double *p, int64_t n,
                           const double *sc, bool first, hipStream_t s)
{
    hipLaunchKernelGGL(update_p_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                       z, p, n, sc, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_update_xr(double *x, double *r, const double *p,
                            const double *ap, int64_t n, double *sc,
                            double *partials, int iter, hipStream_t s)
{
    hipLaunchKernelGGL(update_xr_kernel, dim3(blocks_for(n, 256, kRedBlocks)),
                       dim3(256), 0, s, x, r, p, ap, n, sc, partials,
                       counter_of(partials), iter);
    return hipGetLastError();
}

}  // namespace m2s
