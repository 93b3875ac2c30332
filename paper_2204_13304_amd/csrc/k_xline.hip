// k_xline.hip -- the 27-point Gauss-Seidel half-sweep with the x-line
// recurrence solved by a parallel affine scan: a reassociated variant of the
// exact lexicographic sweep (the dependence structure of Sec. 7.2.1's
// 27-point SymGS, scheduled by lines instead of points), for gfx950.
//
// In sweep order, point i of line (j, k) depends on the new value of point
// i - 1 of its own line through x_i = g_i + c x_{i-1}, c = -off / diag,
// where g_i = (r_i - off S_i) / diag collects every other neighbour: the
// new values of plane k - 1 and of line j - 1, the old values of point
// i + 1, of line j + 1 and of plane k + 1.  Whole lines can therefore be
// updated at once: line (j, k) needs line (j - 1, k) and lines j - 1 .. j + 1
// of plane k - 1, i.e. the line schedule T = j + 2k with 3n - 2 steps on an
// n^3 grid (against 7n - 6 point hyperplanes).  Along a line the recurrence
// is a chain of affine maps; it is solved as a chunked prefix scan of those
// maps over the workgroup (each thread composes its chunk of the line, the
// chunk maps are scanned in LDS, each thread replays its chunk from its
// incoming value).  Every chunk before a thread's own holds P full points,
// so its map is x -> c^P x + B and only the offsets B need scanning: with
// shuffles inside each wavefront, then across the four wavefronts' totals
// in LDS.  The scan reassociates the sums, so the result agrees with the
// lexicographic sweep to rounding, not bitwise.
//
// Schedule: a workgroup owns one plane at a time, handed out in increasing
// k by a ticket counter, and walks the plane's lines in order.  The plane
// above reads each new value through a record of the workspace's record
// array -- the value with the launch's epoch beside each half (the boundary
// records of the tile kernels), written once per launch at device scope --
// and polls the records of line j + 1 of the plane below themselves: the
// poll is the data load, with no progress word, fence or store wait.  The
// two lines below that, j - 1 and j, stay in an LDS window from earlier
// steps.  A plane's holder took its ticket before every later plane's, so
// the chain of waits always ends at a running workgroup and no residency
// assumption is needed.
#include "m2s_internal.hpp"
#include "tile_common.hpp"

#include <algorithm>
#include <cstdlib>

namespace m2s {

constexpr int XL_NT = 256;

struct XLArgs {
    Grid g;
    const double *r;
    const double *xin;   // nullptr: start from zero
    double *xout;
    void *rec;           // one record per point, indexed like xout
    double off, inv_diag;
    uint64_t *ticket;
    uint64_t ticket_base;
    unsigned epoch;
    int *err;
    int spin_limit;
};

template <bool BWD>
__global__ void __launch_bounds__(XL_NT) xline_sweep_kernel(XLArgs a)
{
    using R = Rec<double>;
    extern __shared__ double sm[];
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    double *const win = sm;               // plane k - 1: lines mod 3
    double *const prev = sm + 3 * nx;     // new values of line j - 1
    double *const cur = sm + 4 * nx;      // g, then new values, of line j
    __shared__ double s_tot[XL_NT / 64];  // scan: per-wavefront totals
    __shared__ int s_k, s_abort;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int P = (nx + XL_NT - 1) / XL_NT;   // points per thread chunk
    const int i0 = min(nx, tid * P), i1 = min(nx, i0 + P);
    const long plane = (long)nx * ny;
    const long last = plane * nz - 1;
    const double off = a.off, inv_diag = a.inv_diag;
    const double c = -off * inv_diag;
    const unsigned ep = a.epoch;
    const __amdgpu_buffer_rsrc_t rs_rec = __builtin_amdgcn_make_buffer_rsrc(
        a.rec, 0, (int)(unsigned)((plane * nz) * R::bytes), 0x00020000);
    // c^(P 2^b), b = 0 .. 5: the multipliers of the scan's levels (every
    // chunk before a thread's own is full, P points: its map is
    // x -> c^P x + B)
    double cp[6];
    cp[0] = 1.0;
    for (int q = 0; q < P; ++q) cp[0] *= c;
#pragma unroll
    for (int b = 1; b < 6; ++b) cp[b] = cp[b - 1] * cp[b - 1];
    const double c64 = cp[5] * cp[5];     // a whole wavefront's chunks
    double clane = 1.0;                   // c^(P lane)
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (lane & (1 << b)) clane *= cp[b];

    // element (i, j, k) of the sweep's own order; the backward sweep runs
    // the forward one on the point-reflected grid (the operator is
    // symmetric under the reflection)
    auto vidx = [&](int i, int j, int k) -> long {
        const long v = ((long)k * ny + j) * nx + i;
        return BWD ? last - v : v;
    };
    auto inb = [&](int i, int j, int k) {
        return i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
    };
    // new value of plane k - 1, line l (window), 0 outside the grid
    auto wnew = [&](int i, int l) -> double {
        return (i >= 0 && i < nx && l >= 0 && l < ny)
                   ? win[(l % 3) * nx + i]
                   : 0.0;
    };
    if (tid == 0) s_abort = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const uint64_t tk =
                atomicAdd((unsigned long long *)a.ticket, 1ull) - a.ticket_base;
            s_k = (tk < (uint64_t)nz) ? (int)tk : -1;
        }
        __syncthreads();
        const int k = s_k;
        if (k < 0) return;
        for (int e = tid; e < nx; e += XL_NT) prev[e] = 0.0;
        int spin = a.spin_limit;
        for (int j = 0; j < ny; ++j) {
            // r and the old values (plane k + 1, line j + 1, point i + 1)
            // do not depend on the plane below: their loads go out first
            for (int i = tid; i < nx; i += XL_NT) {
                double s = 0.0;
                if (a.xin) {
#pragma unroll
                    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
                        for (int di = -1; di <= 1; ++di) {
                            const int ii = i + di, jj = j + dj;
                            s += inb(ii, jj, k + 1) ? a.xin[vidx(ii, jj, k + 1)]
                                                    : 0.0;
                        }
#pragma unroll
                    for (int di = -1; di <= 1; ++di)
                        s += inb(i + di, j + 1, k)
                                 ? a.xin[vidx(i + di, j + 1, k)]
                                 : 0.0;
                    if (i + 1 < nx) s += a.xin[vidx(i + 1, j, k)];
                }
                cur[i] = a.r[vidx(i, j, k)] - off * s;
            }
            // lines of plane k - 1 entering the window: j + 1 (and line 0
            // at the first step), each point's record polled until it
            // carries this launch's epoch
            if (k > 0) {
                const int l0 = j == 0 ? 0 : j + 1, l1 = min(j + 1, ny - 1);
                for (int l = l0; l <= l1; ++l)
                    for (int i = tid; i < nx; i += XL_NT) {
                        const unsigned off_b =
                            (unsigned)vidx(i, l, k - 1) * R::bytes;
                        typename R::V rv = R::load(rs_rec, off_b);
                        while (!R::ready(rv, ep)) {
                            if (--spin < 0 ||
                                __hip_atomic_load(a.err, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)) {
                                __hip_atomic_fetch_or(
                                    a.err, kErrTimeout, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
                                s_abort = 1;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            rv = R::load(rs_rec, off_b);
                        }
                        win[(l % 3) * nx + i] = R::value(rv);
                    }
            }
            __syncthreads();
            if (s_abort) return;
            // add the new values: plane k - 1 (window) and line j - 1
            for (int i = tid; i < nx; i += XL_NT) {
                double s = 0.0;
                if (k > 0) {
#pragma unroll
                    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
                        for (int di = -1; di <= 1; ++di)
                            s += wnew(i + di, j + dj);
                }
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di;
                    s += (ii >= 0 && ii < nx) ? prev[ii] : 0.0;
                }
                cur[i] = (cur[i] - off * s) * inv_diag;
            }
            __syncthreads();
            // the chunk's offset: x_end = c^len x_before + Bm
            double Bm = 0.0;
            for (int i = i0; i < i1; ++i) Bm = fma(c, Bm, cur[i]);
            // inclusive scan of the offsets over the wavefront's lanes
            double b = Bm;
#pragma unroll
            for (int lv = 0; lv < 6; ++lv) {
                const double o = __shfl_up(b, 1 << lv, 64);
                if (lane >= (1 << lv)) b = fma(cp[lv], o, b);
            }
            double ex = __shfl_up(b, 1, 64);  // lanes before this one
            if (lane == 0) ex = 0.0;
            if (lane == 63) s_tot[wv] = b;
            __syncthreads();
            // x just before this chunk: the earlier wavefronts' chunks,
            // then the earlier lanes'
            double xw = 0.0;
            for (int v = 0; v < wv; ++v) xw = fma(c64, xw, s_tot[v]);
            double xv = fma(clane, xw, ex);
            for (int i = i0; i < i1; ++i) {
                xv = fma(c, xv, cur[i]);
                cur[i] = xv;
            }
            __syncthreads();
            // the line: result, record for the plane above, line window
            for (int i = tid; i < nx; i += XL_NT) {
                const double v = cur[i];
                const long p = vidx(i, j, k);
                a.xout[p] = v;
                if (k + 1 < nz)
                    R::store(rs_rec, (unsigned)p * R::bytes, R::make(v, ep));
                prev[i] = v;
            }
        }
    }
}

size_t xline_lds_bytes(int nx) { return sizeof(double) * 5 * (size_t)nx; }

// Half-sweep xin -> xout of a CONST27 FP64 operator; rec: one 16-byte
// record per point (device memory, any contents: the epoch of this launch
// tells new records from old ones).
hipError_t launch_xline_sweep(const m2s_stencil &A, const void *r,
                              const void *xin, void *xout, bool bwd,
                              Workspace &ws, void *rec, hipStream_t s)
{
    const size_t lds = xline_lds_bytes(A.ext.nx);
    if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              ws.dev) != hipSuccess)
        return hipErrorInvalidValue;
    const int grid = std::max(1, std::min(A.ext.nz, 2 * cus));
    XLArgs a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.r = (const double *)r;
    a.xin = (const double *)xin;
    a.xout = (double *)xout;
    a.rec = rec;
    a.off = A.offdiag;
    a.inv_diag = 1.0 / A.diag;
    a.ticket = ws.ticket;
    a.ticket_base = ws.ticket_base;
    // every workgroup takes one ticket past the last plane
    ws.ticket_base += (uint64_t)A.ext.nz + (uint64_t)grid;
    if (++ws.epoch == 0) ++ws.epoch;
    a.epoch = ws.epoch;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    auto k = bwd ? xline_sweep_kernel<true> : xline_sweep_kernel<false>;
    hipError_t err = hipFuncSetAttribute(
        (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(grid), dim3(XL_NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace m2s
