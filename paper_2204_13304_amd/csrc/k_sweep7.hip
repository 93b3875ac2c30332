// k_sweep7.hip -- the block SSOR half-sweep of the NPB-LU-shaped BLOCK7x5
// operator (7-point stencil, 5 unknowns per point, constant 5x5 blocks;
// Sec. 7.1) as a persistent, tiled wavefront kernel for gfx950.
//
// Schedule.  Point (i, j, k) runs at step T = i + j + k, the hyperplane of
// Eq. (hyperplane) with unit weights (Sec. 6.1.3): the three lower neighbours
// have smaller T.  A tile is 16 consecutive j by KT = 4 * NW consecutive k,
// one lane per row; the lower neighbours of its rows lie in the tile or in
// tiles (j - 1, k) and (j, k - 1) of the tile grid (rectangular tiles are
// acyclic for 7 points).  Tiles are handed out in lexicographic (k-tile,
// j-tile) order from a ticket counter.
//
// Wavefront roles (as in the 27-point kernel): NW compute wavefronts (one
// lane per row, LDS and FP64 only, plus the boundary publication), 2 NW
// memory wavefronts (per compute wavefront one for x -- coalesced 4-column
// windows of x_old in, finished pieces of x out -- and one for b and the
// old-value halo rows; loads are parked 4 steps in registers), one poll
// wavefront (the neighbour tiles' boundary records).  A value written by one
// wavefront in step T is read by another from step T + 1 on.
//  * LDS rings of 8 columns x 5 components per row.  At its front f a row
//    reads its neighbours at column f and its own old value at f and f + 1;
//    x_old is staged in windows [f + 2, f + 6), b in [f + 1, f + 5), and
//    [f - 4, f) is stored, all by the row's memory wavefront at the row's
//    phase of the 4-step cycle (the store read comes before the staging
//    write that reuses its slots).
//  * The arithmetic is b7_combine, shared with the sequential kernel.
//  * Boundary rows (j0 + 15 of every plane, j0 .. j0 + 14 of the top plane)
//    are published per step into a step-major slice of epoch-tagged records,
//    one record per component; consumers poll them 4 steps ahead.
#include "m2s_internal.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace m2s {

constexpr int B7_TJ = 16;    // j-rows per tile
constexpr int B7_RJ = 18;    // ring rows per plane: jj = -1 .. 16
constexpr int B7_W = 8;      // ring columns
constexpr int B7_RS = 41;    // ring row stride (doubles): 8 x 5 + 1
constexpr int B7_POLL = 4;   // boundary poll distance (steps)
constexpr int B7_PRE = 16;   // steps before the smallest row skew

namespace {

// epoch-tagged FP64 record {lo, epoch, hi, epoch}, as in k_sweep27.hip
using Rec4 = __attribute__((ext_vector_type(4))) unsigned;

__device__ __forceinline__ Rec4 rec_make(double v, unsigned ep)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    return Rec4{(unsigned)b, ep, (unsigned)(b >> 32), ep};
}
__device__ __forceinline__ bool rec_ready(Rec4 r, unsigned ep)
{
    return r.y == ep && r.w == ep;
}
__device__ __forceinline__ double rec_value(Rec4 r)
{
    return __builtin_bit_cast(
        double, (unsigned long long)r.x | ((unsigned long long)r.z << 32));
}
__device__ __forceinline__ Rec4 rec_load(__amdgpu_buffer_rsrc_t rs,
                                         unsigned off)
{
    return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 16);
}
__device__ __forceinline__ void rec_store(__amdgpu_buffer_rsrc_t rs,
                                          unsigned off, Rec4 r)
{
    __builtin_amdgcn_raw_buffer_store_b128(r, rs, (int)off, 0, 16);
}
__device__ __forceinline__ double ld64(__amdgpu_buffer_rsrc_t rs,
                                       unsigned off)
{
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
}
__device__ __forceinline__ void st64(__amdgpu_buffer_rsrc_t rs, unsigned off,
                                     double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
        rs, (int)off, 0, 0);
}

}  // namespace

struct B7Args {
    Grid g;
    int ntiles, njt, ns;   // tiles, j-tiles, boundary slices per tile
    const double *b;
    const double *xin;     // nullptr: start from zero
    double *xout;
    double w;
    void *bnd;             // boundary store (records)
    int64_t bnd_elems;     // records
    unsigned epoch;
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

// C: device copy of the block constants.  As a separate read-only,
// non-aliased argument its uniform reads compile to scalar loads.
template <bool BWD, int NW>
__global__ void __launch_bounds__(64 * (3 * NW + 1))
    b7_tile_kernel(B7Args a, const Block7Consts *__restrict__ C)
{
    constexpr int KT = 4 * NW;
    constexpr int NE = KT + 15;          // boundary rows per slice
    constexpr int WB = 5 * NE;           // records per slice
    constexpr int NH = 5 * (KT + 16);    // polled halo records
    constexpr int NRING = (KT + 2) * B7_RJ;
    constexpr int PS = B7_RJ * B7_RS;    // ring plane stride
    constexpr int NT = 64 * (3 * NW + 1);
    constexpr unsigned RB = 16;
    extern __shared__ unsigned char smem_raw[];
    double *const xr = (double *)smem_raw;
    double *const rr = xr + NRING * B7_RS;
    __shared__ int s_tile, s_abort;

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int last = (int)a.g.size() - 1;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int dir = BWD ? -1 : 1;
    const unsigned OOB = 0x80000000u;
    const int nbytes = (int)((unsigned)(last + 1) * 40u);
    const unsigned ep = a.epoch;

    auto xrow = [&](int kq, int jq) -> double * {
        return xr + ((kq + 1) * B7_RJ + (jq + 1)) * B7_RS;
    };
    auto rrow = [&](int kq, int jq) -> double * {
        return rr + (kq * B7_TJ + jq) * B7_RS;
    };
    // element (double) index of virtual column 0, component 0 of row (j, k)
    auto rowbase = [&](int j, int k) -> int {
        const int v = (k * ny + j) * nx;
        return 5 * (BWD ? last - v : v);
    };
    // byte offset of (column c, component q) of a row; OOB outside
    auto boff = [&](bool vrow, int rb, int c, int q) -> unsigned {
        return (vrow && (unsigned)c < (unsigned)nx)
                   ? (unsigned)(rb + dir * 5 * c + q) * 8u
                   : OOB;
    };

    if (tid == 0) s_abort = 0;
    bool aborted = false;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint64_t tk = atomicAdd((unsigned long long *)a.ticket, 1ull) -
                          a.ticket_base;
            s_tile = tk < (uint64_t)a.ntiles ? (int)tk : -1;
        }
        for (int e = tid; e < NRING * B7_RS; e += NT) xr[e] = 0.0;
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0 || aborted) return;
        const int jt = tile % a.njt, vt = tile / a.njt;
        const int j0 = B7_TJ * jt, k0 = KT * vt;
        const int T0 = j0 + k0;
        const int T_start = T0 - 1 - B7_PRE;
        const int T_lastc = T0 + (B7_TJ - 1) + (KT - 1) + nx - 1;
        const int nblk = (T_lastc + 5 - T_start + 15) / 16;

        if (wv < NW) {
            // ================= compute: row (j0 + jj, k0 + kk) =============
            const int jj = l & 15, kk = 4 * wv + (l >> 4);
            const int j = j0 + jj, k = k0 + kk;
            const bool vc = j < ny && k < nz;
            const int sc = j + k;
            double *const own = xrow(kk, jj);
            double *const rown = rrow(kk, jj);
            const int ipub =
                jj == 15 ? kk : (kk == KT - 1 ? KT + jj : -1);
            const bool pub = vc && ipub >= 0;
            const int bout = (vt * a.njt + jt) * a.ns * WB + 5 * ipub - T0 * WB;
            const bool hym = j > 0, hyp = j + 1 < ny, hzm = k > 0,
                       hzp = k + 1 < nz;
            const __amdgpu_buffer_rsrc_t rs_b =
                __builtin_amdgcn_make_buffer_rsrc(
                    a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);
            double xprev[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) xprev[c] = 0.0;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph = 0; ph < 16; ++ph) {
                    const int st = Tb + ph;
                    const int f = st - sc;
                    const int o0 = (f & (B7_W - 1)) * 5;
                    // the block coefficients are read through the scalar
                    // cache every step (an opaque zero offset keeps the
                    // reads in the loop instead of in registers across it)
                    int zc = 0;
                    asm volatile("" : "+s"(zc));
                    const Block7Consts &Cs =
                        *(const Block7Consts *)((const char *)C + zc);
                    const int o1 = ((f + 1) & (B7_W - 1)) * 5;
                    double xq[6][5], bb[5], old[5], res[5];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        xq[0][c] = own[o1 + c];            // +x, old
                        xq[1][c] = own[o0 + B7_RS + c];    // +y, old
                        xq[2][c] = own[o0 + PS + c];       // +z, old
                        xq[3][c] = xprev[c];               // -x, new
                        xq[4][c] = own[o0 - B7_RS + c];    // -y, new
                        xq[5][c] = own[o0 - PS + c];       // -z, new
                        old[c] = own[o0 + c];
                        bb[c] = rown[o0 + c];
                    }
                    const bool has[6] = {f + 1 < nx, hyp, hzp, f > 0, hym,
                                         hzm};
                    b7_combine<BWD>(Cs, a.w, bb, xq, has, old, res);
                    const bool act = vc && (unsigned)f < (unsigned)nx;
                    if (act) {
#pragma unroll
                        for (int c = 0; c < 5; ++c) {
                            own[o0 + c] = res[c];
                            xprev[c] = res[c];
                        }
                    }
                    const int rec = bout + st * WB;
#pragma unroll
                    for (int c = 0; c < 5; ++c)
                        rec_store(rs_b,
                                  act && pub ? (unsigned)(rec + c) * RB : OOB,
                                  rec_make(res[c], ep));
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else if (wv < 3 * NW) {
            // ====== memory wavefronts of compute wavefront m: x (stage
            //        x_old, store finished x) or b (stage b and the
            //        old-value halo rows) ======
            // At step T the 16 rows of plane 4m + (T mod 4) get 4-column
            // windows: lane element e = l + 64q -> row e / 20, column
            // (e % 20) / 5, component e % 5.
            const bool xw_role = wv < 2 * NW;
            const int m = xw_role ? wv - NW : wv - 2 * NW;
            const __amdgpu_buffer_rsrc_t rs_in =
                xw_role ? __builtin_amdgcn_make_buffer_rsrc(
                              (void *)(a.xin ? a.xin : a.b), 0,
                              a.xin ? nbytes : 0, 0x00020000)
                        : __builtin_amdgcn_make_buffer_rsrc(
                              (void *)a.b, 0, nbytes, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_x =
                __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(a.xin ? a.xin : a.b), 0, a.xin ? nbytes : 0,
                    0x00020000);
            const __amdgpu_buffer_rsrc_t rs_o =
                __builtin_amdgcn_make_buffer_rsrc((void *)a.xout, 0, nbytes,
                                                  0x00020000);
            // window start relative to the front: x_old 2, b 1
            const int lead = xw_role ? 2 : 1;
            double pipe[4][5], hpipe[4][2];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
#pragma unroll
                for (int q = 0; q < 5; ++q) pipe[p][q] = 0.0;
                hpipe[p][0] = hpipe[p][1] = 0.0;
            }
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph0 = 0; ph0 < 16; ph0 += 4)
#pragma unroll
                for (int p4 = 0; p4 < 4; ++p4) {
                    const int st = Tb + ph0 + p4;
                    const int kk = 4 * m + p4;
                    if (xw_role) {
                        // all store reads first: a row's window spans two
                        // element groups, and the staging writes below
                        // reuse the slots of the stored columns
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            const int e = l + 64 * q;
                            const int jj = e / 20, o = e % 20;
                            const int cq = o / 5, comp = o % 5;
                            const int j = j0 + jj, k = k0 + kk;
                            const bool v = j < ny && k < nz;
                            const int cs = st - (j + k) - 4 + cq;
                            const double xv =
                                xrow(kk, jj)[(cs & (B7_W - 1)) * 5 + comp];
                            st64(rs_o,
                                 boff(v, v ? rowbase(j, k) : 0, cs, comp), xv);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        const int e = l + 64 * q;
                        const int jj = e / 20, o = e % 20;
                        const int cq = o / 5, comp = o % 5;
                        const int j = j0 + jj, k = k0 + kk;
                        const bool v = j < ny && k < nz;
                        const int c = st - (j + k) + lead + cq;
                        double *const dst =
                            xw_role ? xrow(kk, jj) : rrow(kk, jj);
                        dst[(c & (B7_W - 1)) * 5 + comp] = pipe[p4][q];
                        pipe[p4][q] = ld64(
                            rs_in, boff(v, v ? rowbase(j, k) : 0, c + 4, comp));
                    }
                    if (!xw_role) {
                        // old-value halo rows: (16, 4m + p4) and, for the
                        // last wavefront, plane KT rows 4 p4 .. 4 p4 + 3
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int e = l + 64 * q;
                            const bool isa = e < 20;
                            const bool mine =
                                isa || (m == NW - 1 && e < 100);
                            const int jj = isa ? 16 : 4 * p4 + (e - 20) / 20;
                            const int o = isa ? e : (e - 20) % 20;
                            const int kq = isa ? kk : KT;
                            const int cq = o / 5, comp = o % 5;
                            const int j = j0 + jj, k = k0 + kq;
                            const bool v = mine && j < ny && k < nz;
                            const int cx = st - (j + k) + 2 + cq;
                            if (mine)
                                xrow(kq, jj)[(cx & (B7_W - 1)) * 5 + comp] =
                                    hpipe[p4][q];
                            hpipe[p4][q] = ld64(
                                rs_x,
                                boff(v, v ? rowbase(j, k) : 0, cx + 4, comp));
                        }
                    }
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else {
            // ====== poll wavefront: records l and l + 64 of the halo ======
            // halo row h < KT: (jj = -1, kk = h) from tile (jt - 1, vt),
            // entry h; h = KT + jj: plane k0 - 1 row jj from (jt, vt - 1),
            // entry KT + jj (jj < 15) or KT - 1 (jj = 15)
            int hoff[2], hs[2], hslot[2], hT0[2];
            double *hrow[2];
            bool hv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = l + 64 * q;
                const int h = e / 5, comp = e % 5;
                const bool left = h < KT;
                const int jj = left ? -1 : h - KT;
                const int kk = left ? h : -1;
                const int j = j0 + jj, k = k0 + kk;
                const int pjt = left ? jt - 1 : jt, pvt = left ? vt : vt - 1;
                const int ent = left ? h : (jj < 15 ? KT + jj : KT - 1);
                hv[q] = e < NH && j >= 0 && j < ny && k >= 0 && k < nz;
                hs[q] = j + k;
                hT0[q] = B7_TJ * pjt + KT * pvt;
                hslot[q] = hv[q] ? (pvt * a.njt + pjt) * a.ns * WB + 5 * ent +
                                       comp
                                 : 0;
                hrow[q] = xrow(hv[q] ? kk : 0, hv[q] ? jj : 0) + comp;
                hoff[q] = comp;
            }
            (void)hoff;
            const __amdgpu_buffer_rsrc_t rs_b =
                __builtin_amdgcn_make_buffer_rsrc(
                    a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);
            auto pslice = [&](int q, int T_) -> int {
                const int s = min(max(T_ - hT0[q], 0), a.ns - 1);
                return hslot[q] + s * WB;
            };
            Rec4 ppipe[B7_POLL][2];
#pragma unroll
            for (int p = 0; p < B7_POLL; ++p) ppipe[p][0] = ppipe[p][1] = Rec4{};
            int spin_budget = a.spin_limit;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph0 = 0; ph0 < 16; ph0 += 4)
#pragma unroll
                for (int ph = 0; ph < 4; ++ph) {
                    const int st = Tb + ph0 + ph;
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int c = st - hs[q];
                        if (hv[q] && c >= 0) {
                            double v = 0.0;
                            if (c < nx) {
                                Rec4 r = ppipe[ph & (B7_POLL - 1)][q];
                                const unsigned src =
                                    (unsigned)pslice(q, st) * RB;
                                while (!rec_ready(r, ep)) {
                                    if (--spin_budget < 0 ||
                                        __hip_atomic_load(
                                            a.err, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)) {
                                        __hip_atomic_fetch_or(
                                            a.err, kErrTimeout,
                                            __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
                                        s_abort = 1;
                                        break;
                                    }
                                    __builtin_amdgcn_s_sleep(1);
                                    r = rec_load(rs_b, src);
                                }
                                v = rec_value(r);
                            }
                            hrow[q][(c & (B7_W - 1)) * 5] = v;
                        }
                        ppipe[ph & (B7_POLL - 1)][q] = rec_load(
                            rs_b, hv[q] ? (unsigned)pslice(q, st + B7_POLL) * RB
                                        : OOB);
                    }
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- host --

B7Layout b7_layout(Grid g, int nw)
{
    B7Layout L{};
    L.nw = nw;
    L.kt = 4 * nw;
    L.njt = (g.ny + B7_TJ - 1) / B7_TJ;
    L.nbands = (g.nz + L.kt - 1) / L.kt;
    L.ntiles = L.njt * L.nbands;
    L.ns = g.nx + (B7_TJ - 1) + (L.kt - 1);
    L.wb = 5 * (L.kt + 15);
    L.bnd_elems = (int64_t)L.ntiles * L.ns * L.wb;
    return L;
}

size_t b7_lds_bytes(int nw)
{
    const int kt = 4 * nw;
    return ((size_t)(kt + 2) * B7_RJ + (size_t)kt * B7_TJ) * B7_RS * 8;
}

int b7_threads(int nw) { return 64 * (3 * nw + 1); }

template <bool BWD, int NW>
static hipError_t b7_launch_t(const B7Args &a, const Block7Consts *C,
                              int grid, size_t lds,
                              hipStream_t s)
{
    auto k = b7_tile_kernel<BWD, NW>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
            160 * 1024 - 64);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * (3 * NW + 1)), lds, s, a, C);
    return hipGetLastError();
}

hipError_t launch_sweep7(const m2s_stencil &A, const Block7Consts &C,
                         double omega, const void *b, const void *xin,
                         void *xout, bool bwd, Workspace &ws,
                         const SweepPlan &plan, hipStream_t s)
{
    // device copy of the block constants, refreshed when they change
    if (!ws.b7c) {
        hipError_t e = hipMalloc(&ws.b7c, sizeof(Block7Consts));
        if (e != hipSuccess) return e;
        ws.b7c_valid = false;
    }
    if (!ws.b7c_valid ||
        std::memcmp(&ws.b7c_host, &C, sizeof(Block7Consts)) != 0) {
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpy(ws.b7c, &C, sizeof(Block7Consts),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        std::memcpy(&ws.b7c_host, &C, sizeof(Block7Consts));
        ws.b7c_valid = true;
    }
    const int nw = plan.slab_planes / 4;
    const size_t lds = b7_lds_bytes(nw);
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    if (++ws.epoch == 0) ++ws.epoch;
    B7Args a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.ntiles = plan.nslabs;
    a.njt = ws.tile_nutb;
    a.ns = ws.tile_ns;
    a.b = (const double *)b;
    a.xin = (const double *)xin;
    a.xout = (double *)xout;
    a.w = omega;
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = ws.epoch;
    a.ticket = ws.ticket;
    a.ticket_base = base;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    const Block7Consts *cd = (const Block7Consts *)ws.b7c;
    switch (nw) {
    case 1:
        return bwd ? b7_launch_t<true, 1>(a, cd, plan.grid, lds, s)
                   : b7_launch_t<false, 1>(a, cd, plan.grid, lds, s);
    case 2:
        return bwd ? b7_launch_t<true, 2>(a, cd, plan.grid, lds, s)
                   : b7_launch_t<false, 2>(a, cd, plan.grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace m2s
