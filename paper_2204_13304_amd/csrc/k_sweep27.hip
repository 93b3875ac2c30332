// k_sweep27.hip -- the exact lexicographic Gauss-Seidel half-sweep of the
// 27-point operator (the HPCG SymGS of Sec. 7.1; a Seidel-style stencil,
// Sec. 2.1.2) as a persistent wavefront kernel tuned for gfx950.
//
// Schedule.  A workgroup owns a slab of Bk whole planes; thread (kk, j) owns
// row j of local plane kk and processes column i at local step
// t = i + 2j + 4kk.  Every lower neighbour of a point has a strictly smaller
// t (the hyperplane of Eq. (hyperplane) with weights (1,2,4), Sec. 6.1.3),
// so one workgroup barrier per step orders all in-slab dependences.  Slabs
// are lexicographic intervals, so dependences between slabs only point
// forward; slabs are taken in order from a ticket counter, so a slab only
// ever waits for one that a running workgroup owns.
//
// Data path.
//  * "Current x" rings in LDS: for planes kk = -1 .. Bk and rows -1 .. ny a
//    ring of 16 columns holds the newest value of x (old until the owner
//    updates it, new afterwards) -- the in-place semantics of the paper's
//    Seidel loop, kept only for the columns around each row's front.  Rows
//    -1 and ny and the planes outside the grid stay zero, so the eight
//    neighbour reads of a point need no bounds tests.  Row stride 17 keeps
//    the skewed 64-bit reads of a wave bank-conflict free.  A thread keeps
//    the partial column sums of columns i-1 and i in registers and reads the
//    8 neighbour rows of column i+1 each step.
//  * Old values and r stream from HBM through 8-slot register pipelines
//    (slot = step mod 8, identical for every lane because all rows advance
//    one column per step): a slot is consumed and refilled in the same step,
//    8 steps ahead of use, with clamped always-in-bounds addresses so the
//    loads stay in flight across steps.  Old values are staged into the rings
//    8 columns ahead of the front.
//  * Between slabs the top plane's new values go to a boundary buffer in
//    diagonal layout [i + 2j][j] (i + 2j is the same for every lane at a
//    given step, so both ends are coalesced) that starts filled with a NaN
//    sentinel.  The next slab polls the values themselves -- the data is its
//    own ready flag, one memory round trip, no fences -- stages them just
//    before their first use and resets each entry to the sentinel.  Each
//    slab boundary has its own buffer (a buffer reused within one sweep could
//    be polled by its later consumer before the earlier one reset it).
// The per-point arithmetic is bit-for-bit that of the sequential kernel
// (c27_col / c27_combine association in k_sweep.hip).
#include "m2s_internal.hpp"

#include <algorithm>

namespace m2s {

constexpr int C27_W = 16;     // ring columns
constexpr int C27_WP = 17;    // padded ring stride
constexpr int C27_LEAD = 8;   // own-ring staging lead (columns)
constexpr int C27_U = 8;      // pipeline length = unroll (steps)
constexpr int C27_MAX_THREADS = 512;

template <typename T>
struct BitsOf;
template <>
struct BitsOf<double> {
    using U = unsigned long long;
    static constexpr U sentinel = 0x7FF4000000000BADull;
};
template <>
struct BitsOf<float> {
    using U = unsigned int;
    static constexpr U sentinel = 0x7FA00BADu;
};

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T *p)
{
    using U = typename BitsOf<T>::U;
    U v = __hip_atomic_load((const U *)p, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, v);
}

template <typename T>
__device__ __forceinline__ void st_relaxed(T *p, T v)
{
    using U = typename BitsOf<T>::U;
    __hip_atomic_store((U *)p, __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ bool is_sentinel(T v)
{
    return __builtin_bit_cast(typename BitsOf<T>::U, v) ==
           BitsOf<T>::sentinel;
}

template <typename T>
struct C27Args {
    Grid g;
    int Bk, nslabs;
    const T *r;
    const T *xin;  // nullptr: start from zero
    T *xout;
    T off, inv_diag;
    T *bnd;              // one buffer per slab boundary (nslabs - 1)
    int64_t bnd_stride;  // (nx + 2 ny) * ny
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

template <typename T, bool BWD, bool ZERO>
__global__ void __launch_bounds__(C27_MAX_THREADS)
    c27_slab_kernel(C27Args<T> a)
{
    extern __shared__ unsigned char smem_raw[];
    T *xc = (T *)smem_raw;
    __shared__ int s_slab, s_abort;

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int Bk = a.Bk;
    const int RS = ny + 2;  // ring rows per plane (zero rows -1 and ny)
    const int tid = threadIdx.x;
    const int kk = tid / ny;
    const int j = tid - kk * ny;
    const bool lane_ok = kk < Bk;
    const T zero = T(0);
    const T off = a.off, inv_diag = a.inv_diag;
    // ring of local plane p (-1 .. Bk) and row r (-1 .. ny)
    auto ring = [&](int p, int r) -> T * {
        return xc + ((p + 1) * RS + (r + 1)) * C27_WP;
    };
    // zero the whole ring area once (rows -1 and ny stay zero for ever)
    const int ring_elems = (Bk + 2) * RS * C27_WP;
    for (int e = tid; e < ring_elems; e += blockDim.x) xc[e] = zero;
    if (tid == 0) s_abort = 0;
    __syncthreads();

    // neighbour ring rows: index (dz + 1) * 3 + (dy + 1)
    T *const own = ring(lane_ok ? kk : 0, j);
    T *nb[9];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
            nb[(dz + 1) * 3 + dy + 1] = ring(lane_ok ? kk + dz : 0, j + dy);

    for (;;) {
        if (tid == 0) {
            uint64_t tk = atomicAdd((unsigned long long *)a.ticket, 1ull) -
                          a.ticket_base;
            s_slab = tk < (uint64_t)a.nslabs ? (int)tk : -1;
        }
        __syncthreads();
        const int slab = s_slab;
        if (slab < 0) return;
        const int k0 = slab * Bk;
        const int nbp = min(Bk, nz - k0);  // planes in this slab
        const bool has_prev = k0 > 0;
        const bool has_next = k0 + nbp < nz;
        const bool active = lane_ok && kk < nbp;
        const bool is_bottom = active && kk == 0 && has_prev;
        const bool is_top = active && kk == nbp - 1 && has_next;
        // the ring of plane -1 must read zero on the first slab and the one
        // above the top plane zero on the last slab (an earlier slab of this
        // workgroup may have filled them)
        if (!has_prev)
            for (int e = tid; e < RS * C27_WP; e += blockDim.x) xc[e] = zero;
        if (!has_next)
            for (int e = tid; e < RS * C27_WP; e += blockDim.x)
                xc[(nbp + 1) * RS * C27_WP + e] = zero;
        T *const above = ring(nbp, j);  // plane k0 + nbp (top threads)
        T *const below = ring(-1, j);   // plane k0 - 1 (bottom threads)
        const T *bnd_in =
            a.bnd + (int64_t)(slab > 0 ? slab - 1 : 0) * a.bnd_stride;
        T *bnd_out = a.bnd + (int64_t)slab * a.bnd_stride;
        // global rows of virtual plane kq, row j; a backward sweep walks
        // the reflected row from its end
        const int kv = k0 + (active ? kk : 0);
        const int rj = BWD ? ny - 1 - j : j;
        auto grow = [&](int kq) -> int64_t {
            const int rk = BWD ? nz - 1 - kq : kq;
            return ((int64_t)rk * ny + rj) * nx + (BWD ? nx - 1 : 0);
        };
        const int64_t row_own = grow(kv);
        const int64_t row_up = is_top ? grow(kv + 1) : row_own;
        const int dir = BWD ? -1 : 1;
        // boundary entry of (column i, row j): (i + 2j) * ny + j
        const int64_t bnd_row = 2 * (int64_t)j * ny + j;

        __syncthreads();  // ring zeroing above is complete

        T xo_pipe[C27_U], r_pipe[C27_U], hi_pipe[C27_U], lo_pipe[C27_U];
#pragma unroll
        for (int q = 0; q < C27_U; ++q) {
            xo_pipe[q] = zero; r_pipe[q] = zero;
            hi_pipe[q] = zero; lo_pipe[q] = zero;
        }
        T F_m1 = zero, F_0 = zero, xn_prev = zero;
        int spin_budget = a.spin_limit;

        // own column at step t is i = t - 2j - 4kk; the loop starts early
        // enough to fill every pipeline before column 0 is needed
        const int t_last = (nx - 1) + 2 * (ny - 1) + 4 * (nbp - 1);
        const int t_begin = -(C27_LEAD + C27_U + 8);
        int col = t_begin - 2 * j - 4 * (active ? kk : 0);
        auto clampc = [&](int c) -> int { return min(max(c, 0), nx - 1); };

        bool aborted = false;
        for (int tb = t_begin; tb <= t_last && !aborted; tb += C27_U) {
#pragma unroll
            for (int tau = 0; tau < C27_U; ++tau) {
                // ---- stage old / boundary values into the rings ----
                // (unconditional: columns outside [0, nx) land in ring slots
                // that are dead or never read)
                if (active) {
                    own[(col + C27_LEAD) & (C27_W - 1)] =
                        ZERO ? zero : xo_pipe[tau];
                    if (is_top)
                        above[(col - 4 + C27_LEAD) & (C27_W - 1)] =
                            ZERO ? zero : hi_pipe[tau];
                    if (is_bottom) {
                        // plane -1 column cb is first read one step later
                        const int cb = col + 4;
                        T v = lo_pipe[tau];
                        if (cb >= 0 && cb < nx) {
                            T *src = (T *)bnd_in + bnd_row + (int64_t)cb * ny;
                            while (is_sentinel(v)) {
                                if (--spin_budget < 0 ||
                                    __hip_atomic_load(
                                        a.err, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)) {
                                    __hip_atomic_fetch_or(
                                        a.err, kErrTimeout, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
                                    s_abort = 1;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                                v = ld_relaxed(src);
                            }
                            st_relaxed(src, __builtin_bit_cast(
                                                T, BitsOf<T>::sentinel));
                        }
                        below[cb & (C27_W - 1)] = v;
                    }
                }
                // ---- compute the point at column col ----
                if (active && col >= 0 && col < nx) {
                    const int c = col + 1;
                    const int cw = c & (C27_W - 1);
                    // F'(c): the 8 values of column c outside the row
                    const T v0 = nb[0][cw], v1 = nb[1][cw], v2 = nb[2][cw];
                    const T v3 = nb[3][cw], v4 = nb[5][cw];
                    const T v5 = nb[6][cw], v6 = nb[7][cw], v7 = nb[8][cw];
                    const T xon_r = own[cw];
                    const T Fp = ((v0 + v1) + (v2 + v3)) +
                                 ((v4 + v5) + (v6 + v7));
                    const bool in = c < nx;
                    const T F_p1 = in ? Fp : zero;
                    const T xon = in ? xon_r : zero;
                    if (col == 0) {
                        const T u0 = nb[0][0], u1 = nb[1][0], u2 = nb[2][0];
                        const T u3 = nb[3][0], u4 = nb[5][0];
                        const T u5 = nb[6][0], u6 = nb[7][0], u7 = nb[8][0];
                        F_m1 = zero;
                        F_0 = ((u0 + u1) + (u2 + u3)) + ((u4 + u5) + (u6 + u7));
                        xn_prev = zero;
                    }
                    const T S = (F_m1 + F_0) + (F_p1 + xon);
                    T tt = fma(-off, S, r_pipe[tau]);
                    tt = fma(-off, xn_prev, tt);
                    const T xnew = tt * inv_diag;
                    own[col & (C27_W - 1)] = xnew;
                    a.xout[row_own + dir * col] = xnew;
                    if (is_top)
                        st_relaxed(bnd_out + bnd_row + (int64_t)col * ny,
                                   xnew);
                    F_m1 = F_0;
                    F_0 = F_p1;
                    xn_prev = xnew;
                }
                // ---- refill the consumed pipeline slots, U steps ahead ----
                {
                    if (!ZERO)
                        xo_pipe[tau] =
                            a.xin[row_own +
                                  dir * clampc(col + C27_U + C27_LEAD)];
                    r_pipe[tau] = a.r[row_own + dir * clampc(col + C27_U)];
                    if (!ZERO)
                        hi_pipe[tau] =
                            a.xin[row_up +
                                  dir * clampc(col - 4 + C27_U + C27_LEAD)];
                    lo_pipe[tau] = ld_relaxed(
                        bnd_in +
                        (is_bottom ? bnd_row + (int64_t)clampc(col + 4 + C27_U) *
                                                   ny
                                   : 0));
                }
                ++col;
                __syncthreads();
            }
            aborted = s_abort != 0;
        }
        if (aborted) return;
        __syncthreads();
    }
}

// Fill boundary buffers with the sentinel pattern.
template <typename T>
__global__ void __launch_bounds__(256)
    fill_sentinel_kernel(T *p, int64_t n)
{
    using U = typename BitsOf<T>::U;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        ((U *)p)[q] = BitsOf<T>::sentinel;
}

int c27_max_threads() { return C27_MAX_THREADS; }

int64_t c27_bnd_stride(int nx, int ny) { return (int64_t)(nx + 2 * ny) * ny; }

size_t c27_lds_bytes(int Bk, int ny, m2s_dtype t)
{
    return (size_t)(Bk + 2) * (ny + 2) * C27_WP * (t == M2S_F64 ? 8 : 4);
}

hipError_t c27_fill_sentinel(void *p, m2s_dtype t, int64_t n, hipStream_t s)
{
    int nb = (int)std::min<int64_t>((n + 255) / 256, 8192);
    if (nb < 1) nb = 1;
    if (t == M2S_F64)
        hipLaunchKernelGGL(fill_sentinel_kernel<double>, dim3(nb), dim3(256),
                           0, s, (double *)p, n);
    else
        hipLaunchKernelGGL(fill_sentinel_kernel<float>, dim3(nb), dim3(256),
                           0, s, (float *)p, n);
    return hipGetLastError();
}

template <typename T, bool BWD, bool ZERO>
static hipError_t c27_launch_t(const C27Args<T> &a, int threads, int grid,
                               size_t lds, hipStream_t s)
{
    auto k = c27_slab_kernel<T, BWD, ZERO>;
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

int c27_max_blocks_per_cu(m2s_dtype t, int threads, size_t lds)
{
    int n = 0;
    hipError_t e;
    if (t == M2S_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, c27_slab_kernel<double, false, false>, threads, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, c27_slab_kernel<float, false, false>, threads, lds);
    if (e != hipSuccess || n < 1) n = 1;
    return n;
}

hipError_t launch_sweep27(const m2s_stencil &A, const void *r,
                          const void *xin, void *xout, bool bwd,
                          Workspace &ws, const SweepPlan &plan, hipStream_t s)
{
    const size_t lds = c27_lds_bytes(plan.slab_planes, A.ext.ny, A.dtype);
    // this launch takes tickets [base, base + nslabs + grid)
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    auto fill = [&](auto &a) {
        a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
        a.Bk = plan.slab_planes;
        a.nslabs = plan.nslabs;
        a.bnd_stride = c27_bnd_stride(A.ext.nx, A.ext.ny);
        a.ticket = ws.ticket;
        a.ticket_base = base;
        a.err = ws.err;
        const char *e = getenv("M2S_SPIN_LIMIT");
        a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    };
    const bool zero = xin == nullptr;
    if (A.dtype == M2S_F64) {
        C27Args<double> a{};
        fill(a);
        a.r = (const double *)r;
        a.xin = (const double *)xin;
        a.xout = (double *)xout;
        a.off = A.offdiag;
        a.inv_diag = 1.0 / A.diag;
        a.bnd = (double *)ws.bnd;
        if (bwd)
            return zero ? c27_launch_t<double, true, true>(a, plan.threads,
                                                           plan.grid, lds, s)
                        : c27_launch_t<double, true, false>(a, plan.threads,
                                                            plan.grid, lds, s);
        return zero ? c27_launch_t<double, false, true>(a, plan.threads,
                                                        plan.grid, lds, s)
                    : c27_launch_t<double, false, false>(a, plan.threads,
                                                         plan.grid, lds, s);
    }
    C27Args<float> a{};
    fill(a);
    a.r = (const float *)r;
    a.xin = (const float *)xin;
    a.xout = (float *)xout;
    a.off = (float)A.offdiag;
    a.inv_diag = (float)(1.0 / A.diag);
    a.bnd = (float *)ws.bnd;
    if (bwd)
        return zero ? c27_launch_t<float, true, true>(a, plan.threads,
                                                      plan.grid, lds, s)
                    : c27_launch_t<float, true, false>(a, plan.threads,
                                                       plan.grid, lds, s);
    return zero ? c27_launch_t<float, false, true>(a, plan.threads, plan.grid,
                                                   lds, s)
                : c27_launch_t<float, false, false>(a, plan.threads, plan.grid,
                                                    lds, s);
}

}  // namespace m2s
