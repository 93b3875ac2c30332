// k_sweep.hip -- exact lexicographic Gauss-Seidel / block-SSOR half-sweeps
// (the Seidel-style stencils of the paper, Sec. 2.1.2 and Sec. 4.3.3) as a
// persistent wavefront kernel for gfx950, plus the one-thread sequential
// reference kernel built from the same per-point arithmetic.
//
// Schedule.  The grid is cut into slabs of `Bk` whole planes (lexicographic
// intervals, so every dependence between slabs points from a lower slab to
// a higher one -- the GPU counterpart of SewTh's rule that partitions follow
// the sequential order, Sec. 6.1.1).  Slabs are handed to workgroups through
// a ticket counter in increasing order, so a workgroup only ever waits for a
// slab that a running workgroup already owns (deadlock freedom, the
// argument of Sec. 6.1.1 for crossing dependences).  Inside a slab one
// thread owns one row slot of one plane and walks its row along x; row j of
// local plane kk processes column i at local step
//      t = i + LJ*j + LK*kk      (LJ, LK) = (2, 4) for 27 points,
//                                           (1, 1) for 7 points,
// the thread-partitioning hyperplane of Eq. (hyperplane) with unit
// partitions; every lower neighbour has a strictly smaller t (checked on the
// CPU by the schedule tests).  One workgroup barrier per step orders the
// steps.  Between slabs a monotone progress counter per slab, tagged with
// the launch epoch (never reset), is published with release semantics every
// `G` steps and waited on with acquire semantics -- one counter per
// producer/consumer pair suffices because compacted crossing dependences
// are ordered alike on both ends (Thm. 2, Sec. 6.1.2).
//
// Data path.  Half-sweeps are out of place: new values go to x_out, so a
// point reads its lower (already updated) neighbours from x_out and its
// upper neighbours from x_in; there is no write-after-read hazard and the
// result equals the in-place lexicographic sweep exactly.
#include "m2s_internal.hpp"

#include <algorithm>

namespace m2s {

// --------------------------------------------------------------------------
// Per-point arithmetic (identical in the wavefront and sequential kernels).
// xn: array holding updated values (x_out); xo: values before the sweep
// (x_in, or nullptr for an all-zero start).  Coordinates are virtual.
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld(const T *a, int64_t q)
{
    return a ? a[q] : T(0);
}

// CONST27 column sums for the row (j, k).  The 8 values of column c outside
// the row: v0 (j-1,k-1), v1 (j,k-1), v2 (j+1,k-1), v3 (j-1,k), v4 (j+1,k),
// v5 (j-1,k+1), v6 (j,k+1), v7 (j+1,k+1), zero outside the grid.  In a
// forward sweep v2 and v3 of column i + 1 are the values updated just
// before point i (the tiled kernel reads them last), so the sum is split
// into A(c) = ((v0 + v1) + (v4 + v5)) + (v6 + v7) and D(c) = v2 + v3, and
// F(c) = A(c) + D(c).
template <typename T, bool BWD>
__device__ __forceinline__ void c27_col(const Virt<BWD> &V, const T *xn,
                                        const T *xo, int c, int j, int k,
                                        T &A, T &D)
{
    const Grid &g = V.g;
    if (c < 0 || c >= g.nx) {
        A = D = T(0);
        return;
    }
    const bool jm = j > 0, jp = j < g.ny - 1, km = k > 0, kp = k < g.nz - 1;
    T v0 = (km && jm) ? xn[V.idx(c, j - 1, k - 1)] : T(0);
    T v1 = km ? xn[V.idx(c, j, k - 1)] : T(0);
    T v2 = (km && jp) ? xn[V.idx(c, j + 1, k - 1)] : T(0);
    T v3 = jm ? xn[V.idx(c, j - 1, k)] : T(0);
    T v4 = jp ? ld(xo, V.idx(c, j + 1, k)) : T(0);
    T v5 = (kp && jm) ? ld(xo, V.idx(c, j - 1, k + 1)) : T(0);
    T v6 = kp ? ld(xo, V.idx(c, j, k + 1)) : T(0);
    T v7 = (kp && jp) ? ld(xo, V.idx(c, j + 1, k + 1)) : T(0);
    A = ((v0 + v1) + (v4 + v5)) + (v6 + v7);
    D = v2 + v3;
}

template <typename T, bool BWD>
__device__ __forceinline__ T c27_point(const Virt<BWD> &V, const T *r,
                                       const T *xn, const T *xo, int i, int j,
                                       int k, T off, T inv_diag)
{
    const Grid &g = V.g;
    T Am, Dm, A0, D0, Ap, Dp;
    c27_col<T, BWD>(V, xn, xo, i - 1, j, k, Am, Dm);
    c27_col<T, BWD>(V, xn, xo, i, j, k, A0, D0);
    c27_col<T, BWD>(V, xn, xo, i + 1, j, k, Ap, Dp);
    const T xon = (i < g.nx - 1) ? ld(xo, V.idx(i + 1, j, k)) : T(0);
    const T xnp = (i > 0) ? xn[V.idx(i - 1, j, k)] : T(0);
    const T B = ((Am + Dm) + (A0 + D0)) + (Ap + xon);
    return c27_combine(r[V.idx(i, j, k)], B, Dp, xnp, off, inv_diag);
}

// VAR7: x_p = (r_p + sum_d k_d x_q) / (sum_d k_d), real directions in the
// order -x,+x,-y,+y,-z,+z.  A real-lower neighbour is already updated in a
// forward sweep and not yet updated in a backward one.
template <typename T, bool BWD>
__device__ __forceinline__ T v7_point(const Virt<BWD> &V, const Faces &F,
                                      const T *kx, const T *ky, const T *kz,
                                      const T *r, const T *xn, const T *xo,
                                      int iv, int jv, int kv)
{
    const Grid &g = V.g;
    const int i = V.ri(iv), j = V.rj(jv), k = V.rk(kv);
    const T *lo = BWD ? xo : xn;  // array holding real-lower neighbours
    const T *hi = BWD ? xn : xo;  // array holding real-upper neighbours
    const T kxm = kx[F.ix(i, j, k)], kxp = kx[F.ix(i + 1, j, k)];
    const T kym = ky[F.iy(i, j, k)], kyp = ky[F.iy(i, j + 1, k)];
    const T kzm = kz[F.iz(i, j, k)], kzp = kz[F.iz(i, j, k + 1)];
    const T vmx = i > 0 ? ld(lo, g.idx(i - 1, j, k)) : T(0);
    const T vpx = i < g.nx - 1 ? ld(hi, g.idx(i + 1, j, k)) : T(0);
    const T vmy = j > 0 ? ld(lo, g.idx(i, j - 1, k)) : T(0);
    const T vpy = j < g.ny - 1 ? ld(hi, g.idx(i, j + 1, k)) : T(0);
    const T vmz = k > 0 ? ld(lo, g.idx(i, j, k - 1)) : T(0);
    const T vpz = k < g.nz - 1 ? ld(hi, g.idx(i, j, k + 1)) : T(0);
    T s1 = fma(kxm, vmx, kxp * vpx);
    T s2 = fma(kym, vmy, kyp * vpy);
    T s3 = fma(kzm, vmz, kzp * vpz);
    T S = (s1 + s2) + s3;
    T d = ((kxm + kxp) + (kym + kyp)) + (kzm + kzp);
    return (r[g.idx(i, j, k)] + S) / d;
}

// BLOCK7: x_p <- (1-w) x_p + w B0^{-1} (b_p - sum_{d=1..6} B_d x_{p+d}).
// B0^{-1} through the LU factors with partial pivoting.
template <bool BWD>
__device__ __forceinline__ void b7_point(const Virt<BWD> &V,
                                         const Block7Consts &C, double w,
                                         const double *b, const double *xn,
                                         const double *xo, double *out,
                                         int iv, int jv, int kv)
{
    // sweep coordinates: (iv, jv, kv) - 1 are updated, + 1 are not
    const Grid &g = V.g;
    const int64_t p = V.idx(iv, jv, kv);
    const int di[6] = {1, 0, 0, -1, 0, 0};
    const int dj[6] = {0, 1, 0, 0, -1, 0};
    const int dk[6] = {0, 0, 1, 0, 0, -1};
    double xq[6][5], bb[5], old[5], res[5];
    bool has[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) {
        const int ii = iv + di[v], jj = jv + dj[v], kk = kv + dk[v];
        has[v] = g.in(ii, jj, kk);
        const double *src = v < 3 ? xo : xn;
        const int64_t q = has[v] ? 5 * V.idx(ii, jj, kk) : 0;
#pragma unroll
        for (int c = 0; c < 5; ++c)
            xq[v][c] = (has[v] && src) ? src[q + c] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        bb[a] = b[5 * p + a];
        old[a] = xo ? xo[5 * p + a] : 0.0;
    }
    b7_combine<BWD>(C, w, bb, xq, has, old, res);
#pragma unroll
    for (int a = 0; a < 5; ++a) out[5 * p + a] = res[a];
}

// --------------------------------------------------------------------------
// Kernel arguments.
// --------------------------------------------------------------------------
template <typename T>
struct SweepArgs {
    Grid g;
    SweepPlan plan;
    const T *r;
    const T *xin;   // nullptr: start from zero
    T *xout;
    // CONST27
    T off, inv_diag;
    // VAR7
    const T *kx, *ky, *kz;
    // progress protocol
    uint64_t *flags;
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    uint32_t epoch;
    int spin_limit;
};

enum { KIND_C27 = 0, KIND_V7 = 1, KIND_B7 = 2 };

template <int KIND, typename T, bool BWD>
__device__ __forceinline__ void do_point(const SweepArgs<T> &a,
                                         const Block7Consts &b7, double w,
                                         int iv, int jv, int kv)
{
    Virt<BWD> V{a.g};
    if constexpr (KIND == KIND_C27) {
        a.xout[V.idx(iv, jv, kv)] = c27_point<T, BWD>(
            V, a.r, a.xout, a.xin, iv, jv, kv, a.off, a.inv_diag);
    } else if constexpr (KIND == KIND_V7) {
        Faces F{a.g.nx, a.g.ny, a.g.nz};
        const int i = V.ri(iv), j = V.rj(jv), k = V.rk(kv);
        a.xout[a.g.idx(i, j, k)] = v7_point<T, BWD>(
            V, F, a.kx, a.ky, a.kz, a.r, a.xout, a.xin, iv, jv, kv);
    } else {
        b7_point<BWD>(V, b7, w, (const double *)a.r, (const double *)a.xout,
                      (const double *)a.xin, (double *)a.xout, iv, jv, kv);
    }
}

// Bounded wait until *flag >= want; returns false on timeout or when
// another workgroup has latched an error.
__device__ bool wait_flag(const uint64_t *flag, uint64_t want, int *err,
                          int spin_limit)
{
    for (int n = 0;; ++n) {
        uint64_t v = __hip_atomic_load(flag, __ATOMIC_ACQUIRE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        if (v >= want) return true;
        if ((n & 63) == 63) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT))
                return false;
        }
        if (n >= spin_limit) {
            __hip_atomic_fetch_or(err, kErrTimeout, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int KIND, typename T, bool BWD>
__global__ void __launch_bounds__(1024)
    sweep_wave_kernel(SweepArgs<T> a, Block7Consts b7, double w)
{
    __shared__ int s_slab;
    __shared__ int s_abort;
    const int tid = threadIdx.x;
    const SweepPlan &P = a.plan;
    const int R = P.row_slots, Bk = P.slab_planes, LJ = P.lag_row,
              LK = P.lag_plane, G = P.publish_every;
    const int kk = tid / R, sl = tid - (tid / R) * R;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const uint64_t tag = (uint64_t)a.epoch << 32;
    // steps a neighbour slab must have completed beyond our step t
    const int D = 1 + P.halo_x + LJ * P.halo_y + LK * (Bk - 1);
    if (tid == 0) s_abort = 0;
    for (;;) {
        if (tid == 0) {
            uint64_t tk = atomicAdd((unsigned long long *)a.ticket, 1ull) -
                          a.ticket_base;
            s_slab = tk < (uint64_t)P.nslabs ? (int)tk : -1;
        }
        __syncthreads();
        const int slab = s_slab;
        if (slab < 0) return;
        const int k0 = slab * Bk;
        const int nb = min(Bk, nz - k0);
        const int Tn = nx + LJ * (ny - 1) + LK * (nb - 1);
        const int Tprev = nx + LJ * (ny - 1) + LK * (Bk - 1);
        for (int t = 0; t < Tn; ++t) {
            if (slab > 0 && (t % G) == 0) {
                if (tid == 0) {
                    const int need = min(Tprev, t + G - 1 + D);
                    if (!wait_flag(a.flags + slab - 1, tag | (uint64_t)need,
                                   a.err, a.spin_limit))
                        s_abort = 1;
                }
                __syncthreads();
                if (s_abort) return;
            }
            if (kk < nb) {
                const int rel = t - LK * kk - LJ * sl;
                if (rel >= 0) {
                    // rows s, s+R, ... of this slot start LJ*R steps apart;
                    // with one row per slot (R == ny) there is no wrap
                    const int m = R >= ny ? 0 : rel / (LJ * R);
                    const int i = rel - m * LJ * R;
                    const int j = sl + m * R;
                    if (i < nx && j < ny)
                        do_point<KIND, T, BWD>(a, b7, w, i, j, k0 + kk);
                }
            }
            __syncthreads();
            if (tid == 0 && (((t + 1) % G) == 0 || t + 1 == Tn))
                __hip_atomic_store(a.flags + slab, tag | (uint64_t)(t + 1),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One thread, plain lexicographic order, in place (xn == xo == x).
template <int KIND, typename T, bool BWD>
__global__ void sweep_sequential_kernel(SweepArgs<T> a, Block7Consts b7,
                                        double w)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    a.xin = a.xout;
    for (int kv = 0; kv < a.g.nz; ++kv)
        for (int jv = 0; jv < a.g.ny; ++jv)
            for (int iv = 0; iv < a.g.nx; ++iv)
                do_point<KIND, T, BWD>(a, b7, w, iv, jv, kv);
}

// --------------------------------------------------------------------------
// Host launchers.
// --------------------------------------------------------------------------
static int spin_limit_from_env()
{
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("M2S_SPIN_LIMIT");
        v = e ? std::max(1, atoi(e)) : (1 << 22);
    }
    return v;
}

template <int KIND, typename T>
static hipError_t launch_typed(const m2s_stencil &A, const Block7Consts *b7,
                               double w, const void *r, const void *xin,
                               void *xout, bool bwd, Workspace &ws,
                               const SweepPlan &plan, hipStream_t s)
{
    SweepArgs<T> a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.plan = plan;
    a.r = (const T *)r;
    a.xin = (const T *)xin;
    a.xout = (T *)xout;
    a.off = (T)A.offdiag;
    a.inv_diag = (T)(1.0 / A.diag);
    a.kx = (const T *)A.kx;
    a.ky = (const T *)A.ky;
    a.kz = (const T *)A.kz;
    a.flags = ws.flags;
    a.ticket = ws.ticket;
    a.ticket_base = ws.ticket_base;
    a.err = ws.err;
    a.epoch = ++ws.epoch;
    a.spin_limit = spin_limit_from_env();
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    Block7Consts bc{};
    if (b7) bc = *b7;
    dim3 grid(plan.grid), block(plan.threads);
    if (bwd)
        hipLaunchKernelGGL((sweep_wave_kernel<KIND, T, true>), grid, block, 0,
                           s, a, bc, w);
    else
        hipLaunchKernelGGL((sweep_wave_kernel<KIND, T, false>), grid, block,
                           0, s, a, bc, w);
    return hipGetLastError();
}

hipError_t launch_sweep(const m2s_stencil &A, const Block7Consts *b7,
                        double omega, const void *r, const void *xin,
                        void *xout, bool bwd, bool zero_init, Workspace &ws,
                        const SweepPlan &plan, hipStream_t s)
{
    if (zero_init) xin = nullptr;
    switch (A.kind) {
    case M2S_CONST27:
        return launch_sweep27(A, r, xin, xout, bwd, ws, plan, s);
    case M2S_VAR7:
        return A.dtype == M2S_F64
                   ? launch_typed<KIND_V7, double>(A, b7, omega, r, xin, xout,
                                                   bwd, ws, plan, s)
                   : launch_typed<KIND_V7, float>(A, b7, omega, r, xin, xout,
                                                  bwd, ws, plan, s);
    case M2S_BLOCK7_5:
        if (!b7) return hipErrorInvalidValue;
        return launch_sweep7(A, *b7, omega, r, xin, xout, bwd, ws, plan, s);
    }
    return hipErrorInvalidValue;
}

template <int KIND, typename T>
static hipError_t launch_seq_typed(const m2s_stencil &A,
                                   const Block7Consts *b7, double w,
                                   const void *r, void *x, bool bwd,
                                   hipStream_t s)
{
    SweepArgs<T> a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.r = (const T *)r;
    a.xin = (const T *)x;
    a.xout = (T *)x;
    a.off = (T)A.offdiag;
    a.inv_diag = (T)(1.0 / A.diag);
    a.kx = (const T *)A.kx;
    a.ky = (const T *)A.ky;
    a.kz = (const T *)A.kz;
    Block7Consts bc{};
    if (b7) bc = *b7;
    if (bwd)
        hipLaunchKernelGGL((sweep_sequential_kernel<KIND, T, true>), dim3(1),
                           dim3(64), 0, s, a, bc, w);
    else
        hipLaunchKernelGGL((sweep_sequential_kernel<KIND, T, false>), dim3(1),
                           dim3(64), 0, s, a, bc, w);
    return hipGetLastError();
}

hipError_t launch_sweep_sequential_b7(const m2s_stencil &A,
                                      const Block7Consts &b7, double omega,
                                      const void *b, void *x, bool bwd,
                                      hipStream_t s)
{
    return launch_seq_typed<KIND_B7, double>(A, &b7, omega, b, x, bwd, s);
}

hipError_t launch_sweep_sequential(const m2s_stencil &A, const void *r,
                                   void *x, bool bwd, hipStream_t s)
{
    switch (A.kind) {
    case M2S_CONST27:
        return A.dtype == M2S_F64
                   ? launch_seq_typed<KIND_C27, double>(A, nullptr, 1.0, r, x,
                                                        bwd, s)
                   : launch_seq_typed<KIND_C27, float>(A, nullptr, 1.0, r, x,
                                                       bwd, s);
    case M2S_VAR7:
        return A.dtype == M2S_F64
                   ? launch_seq_typed<KIND_V7, double>(A, nullptr, 1.0, r, x,
                                                       bwd, s)
                   : launch_seq_typed<KIND_V7, float>(A, nullptr, 1.0, r, x,
                                                      bwd, s);
    default:
        return hipErrorInvalidValue;
    }
}

// Occupancy query used by the planner.
int sweep_max_blocks_per_cu(m2s_kind kind, m2s_dtype t, int threads)
{
    int n = 0;
    hipError_t e;
    if (kind == M2S_CONST27 && t == M2S_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, sweep_wave_kernel<KIND_C27, double, false>, threads, 0);
    else if (kind == M2S_CONST27)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, sweep_wave_kernel<KIND_C27, float, false>, threads, 0);
    else if (kind == M2S_VAR7 && t == M2S_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, sweep_wave_kernel<KIND_V7, double, false>, threads, 0);
    else if (kind == M2S_VAR7)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, sweep_wave_kernel<KIND_V7, float, false>, threads, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, sweep_wave_kernel<KIND_B7, double, false>, threads, 0);
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

}  // namespace m2s
