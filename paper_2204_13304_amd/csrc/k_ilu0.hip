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
#include "tile_common.hpp"

#include <algorithm>
#include <cstdlib>

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


// ---------------------------------------------------------------------------
// Band-wavefront triangular solves.  The hyperplane kernels above pay a
// dependent launch per step and touch one cache line per access.  Here a
// workgroup owns a band of KT consecutive planes (all ny rows of each: one
// lane per row, ny * KT <= 512) and walks it on the band's own hyperplanes
// tau = i + 2j + 4kk, kk the plane within the band, with one workgroup
// barrier per step: every lower neighbour of a point is computed 1 to 7
// steps before it, so the new values of the last 8 columns of every row,
// kept in an LDS ring, hold all a point needs.  The plane below the band
// comes from the band below through epoch-tagged records (the value and the
// launch's epoch, one 16-byte record per point of the band's top plane,
// stored once and polled by value); bands are handed out in increasing k by
// a ticket counter, so a band only waits for one a running workgroup owns.
// The upper solve is the lower one on the grid mirrored in i, j and k.
//
// Coefficients are read from a packed copy of the factor laid out by the
// band's step: for plane k and coefficient a, the points of the plane
// diagonal d = i + 2j are stored consecutively by j, so the lanes of a step
// (one plane, consecutive j, i + 2j fixed) load consecutive doubles.
// Of a point's 13 lower neighbours, three are computed one step before it:
// (i + 1, j + 1, k - 1), (i + 1, j - 1, k) and (i - 1, j, k); the other ten
// are summed one step ahead, off the chain of dependent steps.
// ---------------------------------------------------------------------------
constexpr int ILB_RING = 8;     // columns kept per row (lags are 1 .. 7)
constexpr int ILB_MAXT = 512;   // lanes per band (two waves per SIMD: room
                                // for the loads in flight)
constexpr int ILB_PD = 3;       // steps the loads run ahead of their use
constexpr int ILB_POLL = 3;     // steps a record is polled ahead

namespace {

// diagonal d = i + 2j of an nx x ny plane: rows jmin(d) .. jmax(d)
__host__ __device__ inline int ilb_jmin(int d, int nx)
{
    return d - (nx - 1) > 0 ? (d - (nx - 1) + 1) / 2 : 0;
}

}  // namespace

// Packed position q of a plane -> (d, j): the diagonal d is the last one
// whose offset is <= q (doff ascends; empty diagonals share the offset of
// the next one), j = jmin(d) + q - doff[d].
__device__ inline void ilb_locate(const int *__restrict__ doff, int nd,
                                  int nx, int q, int &d, int &j)
{
    int lo = 0, hi = nd - 1;  // doff[lo] <= q < doff[hi] (doff[nd-1] = plane)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (doff[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    d = lo;
    j = ilb_jmin(lo, nx) + (q - doff[lo]);
}

// Packed coefficient arrays: Lp holds 13 arrays of n doubles per plane
// block, Up 14 (the 13 mirrored upper coefficients and 1 / u_pp), at
//   ((k * NA + a) * plane + doff[d] + j - jmin(d)),  d = i + 2j,
// in the logical coordinates of the solve (mirrored for the upper one).
// One thread per packed position (k, q): the diagonal of q gives the point
// (i, j, k) of the lower layout and, mirrored, the point (nx-1-i, ny-1-j,
// nz-1-k) of the upper one; the thread reads each point's contiguous
// coefficients and the lanes of a wavefront write consecutive doubles of
// every array (a thread per point instead wrote every value into its own
// write sector: 4x the stored bytes).
__global__ void __launch_bounds__(256)
    ilu0_pack_kernel(Grid g, const int *__restrict__ doff, int nd,
                     const double *__restrict__ L,
                     const double *__restrict__ U, double *__restrict__ Lp,
                     double *__restrict__ Up)
{
    const int64_t n = g.size();
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; P < n;
         P += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(P / plane);
        const int q = (int)(P - k * plane);
        int d, j;
        ilb_locate(doff, nd, g.nx, q, d, j);
        const int i = d - 2 * j;
        const int64_t pl = ((int64_t)k * g.ny + j) * g.nx + i;
        const int64_t pu = ((int64_t)(g.nz - 1 - k) * g.ny + (g.ny - 1 - j)) *
                               g.nx +
                           (g.nx - 1 - i);
        double lv[13], uv[14];
#pragma unroll
        for (int a = 0; a < 13; ++a) lv[a] = L[13 * pl + a];
#pragma unroll
        for (int a = 0; a < 14; ++a) uv[a] = U[14 * pu + a];
#pragma unroll
        for (int a = 0; a < 13; ++a)
            Lp[((int64_t)k * 13 + a) * plane + q] = lv[a];
        // mirrored lower offset a' of the upper offset m = 26 - a'
#pragma unroll
        for (int a = 0; a < 13; ++a)
            Up[((int64_t)k * 14 + a) * plane + q] = uv[13 - a];
        Up[((int64_t)k * 14 + 13) * plane + q] = 1.0 / uv[0];
    }
}

struct IlbArgs {
    Grid g;                 // extents (the mirrored grid has the same)
    int kt, nbands, nsteps; // planes per band, bands, steps per band
    const int *doff;        // diagonal offsets, nx + 2 ny - 1 entries
    const double *cp;       // packed coefficients (13 or 14 arrays)
    const double *rhs;      // packed; the upper solve reads it reversed
    double *out;            // packed
    void *rec;              // records: (band, column, row), 16 B each
    int64_t rec_elems;
    unsigned epoch;
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

template <bool UPPER>
__global__ void __launch_bounds__(ILB_MAXT) ilu0_band_kernel(IlbArgs a)
{
    using R = Rec<double>;
    constexpr int NA = UPPER ? 14 : 13;
    constexpr unsigned OOB = 0x80000000u;
    extern __shared__ unsigned char smem_raw[];
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz, kt = a.kt;
    const int ND = nx + 2 * ny - 1;
    // per diagonal d: its first packed index minus its first row, so that
    // the packed index of (i, j) in a plane is sdj[i + 2j] + j
    int *const sdj = (int *)smem_raw;
    double *const ring = (double *)(smem_raw + ((ND * 4 + 15) / 16) * 16);
    __shared__ int s_band, s_abort;
    const int t = threadIdx.x;
    const int j = t % ny, kk = t / ny;
    const bool row = kk < kt;
    const int64_t plane = (int64_t)nx * ny;
    const int RW = ny + 2;                // rows -1 .. ny
    const int nring = (kt + 1) * ILB_RING * RW;
    // ring slot of (plane kq in -1 .. kt-1, row jq in -1 .. ny, column c):
    // column-slot major, rows consecutive, so that the lanes of a wave
    // (consecutive rows) read consecutive doubles, free of bank conflicts
    auto rix = [&](int kq, int jq, int c) -> int {
        return ((kq + 1) * ILB_RING + (c & (ILB_RING - 1))) * RW + jq + 1;
    };
    const int64_t nlast = a.g.size() - 1;
    // coefficients through a buffer resource: the lane's offset in a VGPR,
    // the coefficient array's (q * plane * 8) as a scalar offset
    const __amdgpu_buffer_rsrc_t rs_cp = __builtin_amdgcn_make_buffer_rsrc(
        (void *)a.cp, 0, (int)((nlast + 1) * NA * 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs_rec = __builtin_amdgcn_make_buffer_rsrc(
        a.rec, 0, (int)(a.rec_elems * R::bytes), 0x00020000);
    for (int e = t; e < ND; e += blockDim.x)
        sdj[e] = a.doff[e] - ilb_jmin(e, nx);
    if (t == 0) s_abort = 0;
    int spin_budget = a.spin_limit;
    for (;;) {
        __syncthreads();
        if (t == 0) {
            const uint64_t tk =
                atomicAdd((unsigned long long *)a.ticket, 1ull) - a.ticket_base;
            s_band = (tk < (uint64_t)a.nbands && !s_abort) ? (int)tk : -1;
        }
        for (int e = t; e < nring; e += blockDim.x) ring[e] = 0.0;
        __syncthreads();
        const int b = s_band;
        if (b < 0) break;
        const int k0 = b * kt;
        const int k = k0 + kk;
        const bool vrow = row && k < nz;
        // the top plane of every band but the last publishes its values
        const bool pub = vrow && kk == kt - 1 && b + 1 < a.nbands;
        // lanes of plane 0 fetch the band below's top-plane row j
        const bool halo = row && kk == 0 && b > 0;
        // records: 32-bit (the host keeps them below 2^31 bytes)
        const int rbase_out = (b * nx) * ny + j;
        const int rbase_in = ((b - 1) * nx) * ny + j;
        // packed index (within the coefficient array) of the point this
        // lane handles at step s
        // (32-bit: 14 n doubles stay below 2^31 bytes)
        const int kplane = k * (int)plane;
        auto pidx = [&](int s, bool &ok) -> int {
            const int i = s - 2 * j - 4 * kk;
            ok = vrow && i >= 0 && i < nx;
            return ok ? kplane + sdj[s - 4 * kk] + j : 0;
        };
        // loads of step s's point: 13 (14) coefficients and the rhs
        double cf[ILB_PD][NA], rv[ILB_PD];
        typename R::V hrec[ILB_POLL];
        auto issue = [&](int slot, int s) {
            bool ok;
            const int pi = pidx(s, ok);
            // point pi of plane k: coefficient q at (k * NA + q) * plane +
            // (pi - k * plane); a wave with no point at step s skips them
            if (ok) {
                const unsigned vo = (unsigned)(kplane * (NA - 1) + pi) * 8u;
#pragma unroll
                for (int q = 0; q < NA; ++q)
                    cf[slot][q] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(
                                    rs_cp, (int)vo, (int)(q * plane * 8), 0));
                rv[slot] = a.rhs[UPPER ? nlast - pi : pi];
            } else {
#pragma unroll
                for (int q = 0; q < NA; ++q) cf[slot][q] = 0.0;
                rv[slot] = 0.0;
            }
        };
        // the halo column of row j written at step s: c = s - 2j + 4
        auto hpoll = [&](int slot, int s) {
            const int c = s - 2 * j + 4;
            const bool ok = halo && c >= 0 && c < nx;
            hrec[slot] = R::load(
                rs_rec, ok ? (unsigned)((rbase_in + c * ny) *
                                        R::bytes)
                           : OOB);
        };
        // Steps run from S0 = -4: the band below's value of row j, column c
        // is written into the ring at step c + 2j - 4 (one step before the
        // first point that reads it), from column 0 of row 0 on.  Step s
        // of the loop: the point of step s (its late terms), the halo value
        // of step s, the early sum of the point of step s + 1, then the
        // loads of step s + ILB_PD and the poll of step s + ILB_POLL.
        constexpr int S0 = -4;
        double se = 0.0;          // early sum of the next point
        double yprev = 0.0;       // this row's value of the previous column
#pragma unroll
        for (int q = 0; q < ILB_PD; ++q) issue(q, S0 + q);
#pragma unroll
        for (int q = 0; q < ILB_POLL; ++q) hpoll(q, S0 + q);
        // blocks of ILB_PD * ILB_POLL steps keep the rings' slots
        // compile-time: step S0 + m uses slot m mod ILB_PD / ILB_POLL
        constexpr int BLK = ILB_PD * ILB_POLL;
        const int nblk = (a.nsteps - S0 + BLK - 1) / BLK;
        for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
            for (int ph = 0; ph < BLK; ++ph) {
                const int s = S0 + blk * BLK + ph;
                const int cs = ph % ILB_PD;         // slot of step s
                const int cn = (ph + 1) % ILB_PD;   // slot of step s + 1
                const int hs = ph % ILB_POLL;       // poll slot of step s
                // --- the point of step s: three late terms ---------------
                {
                    const int i = s - 2 * j - 4 * kk;
                    if (vrow && i >= 0 && i < nx) {
                        const double *c = cf[cs];
                        // offsets (dk, dj, di): (-1, +1, +1) -> a 8,
                        // (0, -1, +1) -> a 11, (0, 0, -1) -> a 12
                        double sum = se;
                        sum = fma(c[8], ring[rix(kk - 1, j + 1, i + 1)], sum);
                        sum = fma(c[11], ring[rix(kk, j - 1, i + 1)], sum);
                        sum = fma(c[12], yprev, sum);
                        double y = rv[cs] - sum;
                        if (UPPER) y *= c[13];
                        ring[rix(kk, j, i)] = y;
                        yprev = y;
                        bool okp;
                        a.out[pidx(s, okp)] = y;
                        if (pub)
                            R::store(rs_rec,
                                     (unsigned)((rbase_out + i * ny) *
                                                R::bytes),
                                     R::make(y, a.epoch));
                    }
                }
                // --- the band below's top-plane value of step s ------------
                {
                    const int hc = s - 2 * j + 4;
                    if (halo && hc >= 0 && hc < nx) {
                        typename R::V r = hrec[hs];
                        const unsigned src =
                            (unsigned)((rbase_in + hc * ny) *
                                       R::bytes);
                        bool retried = false;
                        while (!R::ready(r, a.epoch)) {
                            retried = true;
                            if (--spin_budget < 0 ||
                                __hip_atomic_load(a.err, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)) {
                                __hip_atomic_fetch_or(
                                    a.err, kErrTimeout, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
                                s_abort = 1;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            r = R::load(rs_rec, src);
                        }
                        ring[rix(-1, j, hc)] = R::value(r);
                        // caught up: the polls issued before the wait were
                        // too early as well
                        if (retried) {
#pragma unroll
                            for (int q = 1; q < ILB_POLL; ++q)
                                hpoll((ph + q) % ILB_POLL, s + q);
                        }
                    }
                }
                // --- the early sum of the point of step s + 1 -------------
                {
                    const int i = s + 1 - 2 * j - 4 * kk;
                    double e = 0.0;
                    if (vrow && i >= 0 && i < nx) {
                        const double *c = cf[cn];
                        // (dk = -1, dj, di) but (-1, +1, +1); then
                        // (0, -1, -1), (0, -1, 0): every one computed at
                        // least two steps before the point
                        // three partial sums keep the chain short
                        double e0 = 0.0, e1 = 0.0, e2;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int dj = q / 3 - 1, di = q % 3 - 1;
                            e0 = fma(c[q], ring[rix(kk - 1, j + dj, i + di)],
                                     e0);
                        }
#pragma unroll
                        for (int q = 4; q < 8; ++q) {
                            const int dj = q / 3 - 1, di = q % 3 - 1;
                            e1 = fma(c[q], ring[rix(kk - 1, j + dj, i + di)],
                                     e1);
                        }
                        e2 = c[9] * ring[rix(kk, j - 1, i - 1)];
                        e2 = fma(c[10], ring[rix(kk, j - 1, i)], e2);
                        e = (e0 + e1) + e2;
                    }
                    se = e;
                }
                // --- loads ahead ------------------------------------------
                issue(cs, s + ILB_PD);
                hpoll(hs, s + ILB_POLL);
                __syncthreads();
            }
            if (s_abort) break;
        }
        if (s_abort) break;
    }
}

// r (natural) into the lower solve's packed order (a thread per packed
// position, gathering, so that the stores are coalesced); z out of the
// upper solve's (the lower order reversed: the mirrored diagonal i' + 2j' is
// the reversed one, its rows in reverse order, the planes reversed; a thread
// per natural point, gathering).
__global__ void __launch_bounds__(256)
    ilu0_pack_vec_kernel(Grid g, const int *__restrict__ doff, int nd,
                         const double *__restrict__ v, double *__restrict__ vp,
                         int unpack_upper)
{
    const int64_t n = g.size();
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; P < n;
         P += (int64_t)gridDim.x * blockDim.x) {
        if (unpack_upper) {
            // P natural; its lower packed position pl, read reversed
            const int i = (int)(P % g.nx);
            const int64_t t = P / g.nx;
            const int j = (int)(t % g.ny), k = (int)(t / g.ny);
            const int d = i + 2 * j;
            const int64_t pl =
                (int64_t)k * plane + doff[d] + j - ilb_jmin(d, g.nx);
            vp[P] = v[n - 1 - pl];
        } else {
            // P packed
            const int k = (int)(P / plane);
            const int q = (int)(P - k * plane);
            int d, j;
            ilb_locate(doff, nd, g.nx, q, d, j);
            vp[P] = v[((int64_t)k * g.ny + j) * g.nx + (d - 2 * j)];
        }
    }
}

// ---------------------------------------------------------------- host --

IlbLayout ilb_layout(const Grid &g)
{
    IlbLayout L{};
    if (g.ny > ILB_MAXT) return L;   // kt = 0: no band kernel for these
    L.kt = std::max(1, std::min(g.nz, ILB_MAXT / g.ny));
    L.nbands = (g.nz + L.kt - 1) / L.kt;
    L.nsteps = (g.nx - 1) + 2 * (g.ny - 1) + 4 * (L.kt - 1) + 1;
    L.threads = ((L.kt * g.ny + 63) / 64) * 64;
    const int nd = g.nx + 2 * g.ny - 1;
    L.doff.resize(nd);
    int acc = 0;
    for (int d = 0; d < nd; ++d) {
        L.doff[d] = acc;
        const int jlo = ilb_jmin(d, g.nx), jhi = std::min(g.ny - 1, d / 2);
        acc += std::max(0, jhi - jlo + 1);
    }
    L.lds = (size_t)((nd * 4 + 15) / 16) * 16 +
            (size_t)(L.kt + 1) * (g.ny + 2) * ILB_RING * 8;
    return L;
}

hipError_t launch_ilu0_pack(const m2s_stencil &A, const int *doff,
                            const double *L, const double *U, double *Lp,
                            double *Up, hipStream_t s)
{
    const Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    const int64_t n = g.size();
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    const int nd = g.nx + 2 * g.ny - 1;
    hipLaunchKernelGGL(ilu0_pack_kernel, dim3(std::max(1, nb)), dim3(256), 0,
                       s, g, doff, nd, L, U, Lp, Up);
    return hipGetLastError();
}

template <bool UPPER>
static hipError_t ilb_launch(const IlbArgs &a, int grid, int threads,
                             size_t lds, hipStream_t s)
{
    auto k = ilu0_band_kernel<UPPER>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
            160 * 1024 - 64);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_ilu0_apply_packed(const m2s_stencil &A, const IlbLayout &L,
                                    const int *doff, const double *Lp,
                                    const double *Up, const double *r,
                                    double *y, double *t, double *z,
                                    Workspace &ws, void *rec,
                                    int64_t rec_elems, hipStream_t s)
{
    const Grid g{A.ext.nx, A.ext.ny, A.ext.nz};
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess)
        return hipErrorInvalidValue;
    const int grid = std::max(1, std::min(L.nbands, cus));
    const int64_t n = g.size();
    const int nb = (int)std::max<int64_t>(
        1, std::min<int64_t>((n + 255) / 256, 8192));
    const char *e = getenv("M2S_SPIN_LIMIT");
    IlbArgs a{};
    a.g = g;
    a.kt = L.kt;
    a.nbands = L.nbands;
    a.nsteps = L.nsteps;
    a.doff = doff;
    a.rec = rec;
    a.rec_elems = rec_elems;
    a.ticket = ws.ticket;
    a.err = ws.err;
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    // r into the lower solve's order (t), lower solve into y, upper solve
    // (reading y backwards) into t, t back into z's natural order
    const int nd = g.nx + 2 * g.ny - 1;
    hipLaunchKernelGGL(ilu0_pack_vec_kernel, dim3(nb), dim3(256), 0, s, g,
                       doff, nd, r, t, 0);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int pass = 0; pass < 2; ++pass) {
        a.ticket_base = ws.ticket_base;
        ws.ticket_base += (uint64_t)L.nbands + (uint64_t)grid;
        if (++ws.epoch == 0) ++ws.epoch;
        a.epoch = ws.epoch;
        if (pass == 0) {
            a.cp = Lp;
            a.rhs = t;
            a.out = y;
            err = ilb_launch<false>(a, grid, L.threads, L.lds, s);
        } else {
            a.cp = Up;
            a.rhs = y;
            a.out = t;
            err = ilb_launch<true>(a, grid, L.threads, L.lds, s);
        }
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(ilu0_pack_vec_kernel, dim3(nb), dim3(256), 0, s, g,
                       doff, nd, t, z, 1);
    return hipGetLastError();
}

}  // namespace m2s
