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
// incoming value).  The scan reassociates the sums, so the result agrees
// with the lexicographic sweep to rounding, not bitwise.
//
// Schedule: a workgroup owns one plane at a time, handed out in increasing
// k by a ticket counter; it walks the plane's lines in order and, after
// each line, publishes the number of lines it has finished.  The workgroup
// of plane k waits (bounded spin) until plane k - 1 has finished line
// j + 1.  The new values and the progress words are written and read at
// device scope, and a line's stores are complete (vmcnt 0 in every wave)
// before its progress word is written, so a reader that sees the word sees
// the line; no cache-wide write-back or invalidation is needed.  A plane's
// holder took its ticket before every later plane's, so the chain of waits
// always ends at a running workgroup and no residency assumption is needed.
#include "m2s_internal.hpp"

#include <algorithm>
#include <cstdlib>

namespace m2s {

constexpr int XL_NT = 256;

struct XLArgs {
    Grid g;
    const double *r;
    const double *xin;   // nullptr: start from zero
    double *xout;
    double off, inv_diag;
    uint64_t *flags;     // per plane: lines finished (cleared per launch)
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

template <bool BWD>
__global__ void __launch_bounds__(XL_NT) xline_sweep_kernel(XLArgs a)
{
    extern __shared__ double sm[];
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    double *const prev = sm;              // new values of line j - 1
    double *const cur = sm + nx;          // g, then new values, of line j
    double *const sA = sm + 2 * nx;       // scan: chunk maps (A, B)
    double *const sB = sA + XL_NT;
    __shared__ int s_k, s_abort;
    const int tid = threadIdx.x;
    const int P = (nx + XL_NT - 1) / XL_NT;   // points per thread chunk
    const int i0 = min(nx, tid * P), i1 = min(nx, i0 + P);
    const long plane = (long)nx * ny;
    const long last = plane * nz - 1;
    const double off = a.off, inv_diag = a.inv_diag;
    const double c = -off * inv_diag;

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

    // values that cross workgroups (the new values of a plane, read by the
    // plane above) are stored and loaded at device scope, so that no cache
    // of another XCD can hold a stale copy; the progress words likewise
    auto load_new = [&](long v) {
        return __hip_atomic_load(a.xout + v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
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
        uint64_t seen = 0;  // thread 0: last progress read of plane k - 1
        for (int j = 0; j < ny; ++j) {
            // r and the old values (plane k + 1, line j + 1, point i + 1)
            // do not depend on the wait: their loads go out first
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
            // plane k - 1 must have finished line j + 1 (or all its lines)
            if (tid == 0 && k > 0) {
                const uint64_t need = (uint64_t)min(j + 2, ny);
                while (seen < need) {
                    seen = __hip_atomic_load(a.flags + (k - 1),
                                             __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                    if (seen >= need) break;
                    if (--spin < 0 ||
                        __hip_atomic_load(a.err, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_fetch_or(a.err, kErrTimeout,
                                              __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __syncthreads();
            if (s_abort) return;
            // add the new values: plane k - 1 (device scope) and line j - 1
            for (int i = tid; i < nx; i += XL_NT) {
                double s = 0.0;
#pragma unroll
                for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
                    for (int di = -1; di <= 1; ++di) {
                        const int ii = i + di, jj = j + dj;
                        s += inb(ii, jj, k - 1) ? load_new(vidx(ii, jj, k - 1))
                                                : 0.0;
                    }
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di;
                    s += (ii >= 0 && ii < nx) ? prev[ii] : 0.0;
                }
                cur[i] = (cur[i] - off * s) * inv_diag;
            }
            __syncthreads();
            // the chunk's map x_end = Am x_before + Bm
            double Am = 1.0, Bm = 0.0;
            for (int i = i0; i < i1; ++i) {
                Am *= c;
                Bm = fma(c, Bm, cur[i]);
            }
            sA[tid] = Am;
            sB[tid] = Bm;
            __syncthreads();
            // inclusive scan of the chunk maps in line order: applying
            // (A1, B1), then (A2, B2), is (A2 A1, A2 B1 + B2)
            for (int d = 1; d < XL_NT; d <<= 1) {
                const double A2 = sA[tid], B2 = sB[tid];
                const double A1 = tid >= d ? sA[tid - d] : 1.0;
                const double B1 = tid >= d ? sB[tid - d] : 0.0;
                __syncthreads();
                sA[tid] = A2 * A1;
                sB[tid] = fma(A2, B1, B2);
                __syncthreads();
            }
            // replay the chunk from x_{i0 - 1} (0 before the line starts)
            double xv = tid > 0 ? sB[tid - 1] : 0.0;
            for (int i = i0; i < i1; ++i) {
                xv = fma(c, xv, cur[i]);
                cur[i] = xv;
            }
            __syncthreads();
            for (int i = tid; i < nx; i += XL_NT) {
                const double v = cur[i];
                __hip_atomic_store(a.xout + vidx(i, j, k), v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                prev[i] = v;
            }
            // every thread's stores have reached device scope before the
            // line is published
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(a.flags + k, (uint64_t)(j + 1),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

size_t xline_lds_bytes(int nx)
{
    return sizeof(double) * (2 * (size_t)nx + 2 * XL_NT);
}

// Half-sweep xin -> xout of a CONST27 FP64 operator; flags: nz zeroed
// 64-bit words of device memory (cleared here, on the stream).
hipError_t launch_xline_sweep(const m2s_stencil &A, const void *r,
                              const void *xin, void *xout, bool bwd,
                              Workspace &ws, uint64_t *flags, hipStream_t s)
{
    const size_t lds = xline_lds_bytes(A.ext.nx);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              ws.dev) != hipSuccess)
        return hipErrorInvalidValue;
    hipError_t err = launch_fill(flags, M2S_F64, A.ext.nz, 0.0, s);
    if (err != hipSuccess) return err;
    const int grid = std::max(1, std::min(A.ext.nz, 2 * cus));
    XLArgs a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.r = (const double *)r;
    a.xin = (const double *)xin;
    a.xout = (double *)xout;
    a.off = A.offdiag;
    a.inv_diag = 1.0 / A.diag;
    a.flags = flags;
    a.ticket = ws.ticket;
    a.ticket_base = ws.ticket_base;
    // every workgroup takes one ticket past the last plane
    ws.ticket_base += (uint64_t)A.ext.nz + (uint64_t)grid;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    auto k = bwd ? xline_sweep_kernel<true> : xline_sweep_kernel<false>;
    err = hipFuncSetAttribute((const void *)k,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k, dim3(grid), dim3(XL_NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace m2s
