// k_sweep7v.hip -- the Gauss-Seidel half-sweep of the VAR7 operator (the
// face-coefficient diffusion stencil of the differentiable solve; 7 points)
// as a persistent, tiled wavefront kernel for gfx950.
//
// Schedule and roles as in the block SSOR kernel.  Point (i, j, k) of the
// (virtual, i.e. sweep-order) grid runs at step T = i + j + k, the
// hyperplane of Eq. (hyperplane) with unit weights (Sec. 6.1.3).  A tile is
// 16 consecutive j by KT = 4 * NW consecutive k, one lane per row; tiles are
// acyclic for 7 points and are handed out in lexicographic (k-tile,
// j-tile) order from a ticket counter.  Roles: NW compute wavefronts (LDS
// and arithmetic only, plus the boundary publication), NW memory
// wavefronts (memory wavefront m stages the data of compute wavefront m's
// rows and stores its finished values), one poll wavefront (the neighbour
// tiles' boundary records).  A value written by one wavefront in step T is
// read by another from step T + 1 on.
//  * Rings of 8 columns per row for x, r and the faces.  At its front f a
//    row needs the faces between itself and its six neighbours.  Per row
//    the ring holds the x-faces in sweep order (face f lies between columns
//    f - 1 and f) and the y- and z-face below the row in sweep order; the
//    faces above are those of the next row and the next plane, so the row
//    j0 + 16 (x and y-faces) and the plane k0 + KT (x and z-faces) are
//    staged as halo.  Face rows on the grid boundary (the row ny, the plane
//    nz in sweep order) are staged too; their rows hold no points.
//  * At step T the rows of plane 4m + (T mod 4) get 4-column windows
//    [f + 2, f + 6) of all five arrays, and [f - 4, f) of x is stored.
//  * The arithmetic is v7_combine, shared with the sequential kernel.
//  * Boundary rows (j0 + 15 of every plane, j0 .. j0 + 14 of the top
//    plane) publish one epoch-tagged record per step; consumers poll them
//    2 or 4 steps ahead (v7_poll).
#include "m2s_internal.hpp"
#include "tile_common.hpp"

#include <algorithm>
#include <cstdlib>

namespace m2s {

constexpr int V7_TJ = 16;    // j-rows per tile
constexpr int V7_RJ = 18;    // x-ring rows per plane: jj = -1 .. 16
constexpr int V7_W = 8;      // ring columns
// Boundary poll distance (steps; a template parameter, 2 or 4): a consumer
// tile settles about POLL steps plus a round trip behind its neighbour, so
// 2 where every tile has a workgroup of its own and crossings are the
// critical path, 4 where tiles queue for workgroups.
inline int v7_poll(int ntiles, int grid) { return ntiles <= grid ? 2 : 4; }
constexpr int V7_PRE = 16;   // steps before the smallest row skew

template <typename T>
struct V7Args {
    Grid g;
    int ntiles, njt, ns;   // tiles, j-tiles, boundary slices per tile
    const T *r;
    const T *xin;          // nullptr: start from zero
    T *xout;
    const T *kx, *ky, *kz;
    void *bnd;             // boundary store (records)
    int64_t bnd_elems;     // records
    unsigned epoch;        // this launch's tag, never 0
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

template <typename T, bool BWD, int NW, int POLL>
__global__ void __launch_bounds__(64 * (2 * NW + 1))
    v7_tile_kernel(V7Args<T> a)
{
    using R = Rec<T>;
    constexpr int KT = 4 * NW;
    constexpr int WB = KT + 15;               // records per slice
    constexpr int NH = KT + 16;               // polled halo rows
    constexpr int NXR = (KT + 2) * V7_RJ;     // x: planes -1..KT, rows -1..16
    constexpr int NRR = KT * V7_TJ;           // r and x-faces
    constexpr int NYR = KT * (V7_TJ + 1);     // y-faces: rows 0..16
    // z-faces: planes 0..KT, (KT + 1) * 16 rows (last, sized on the host)
    constexpr int NT = 64 * (2 * NW + 1);
    constexpr unsigned RB = R::bytes;
    constexpr unsigned ES = sizeof(T);
    extern __shared__ unsigned char smem_raw[];
    T *const xr = (T *)smem_raw;
    T *const rr = xr + NXR * V7_W;
    T *const kxr = rr + NRR * V7_W;
    T *const kyr = kxr + NRR * V7_W;
    T *const kzr = kyr + NYR * V7_W;
    __shared__ int s_tile, s_abort;

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int dir = BWD ? -1 : 1;
    const unsigned OOB = 0x80000000u;
    const unsigned ep = a.epoch;

    auto xrow = [&](int kq, int jq) -> T * {
        return xr + ((kq + 1) * V7_RJ + (jq + 1)) * V7_W;
    };
    auto rrow = [&](int kq, int jq) -> T * {
        return rr + (kq * V7_TJ + jq) * V7_W;
    };
    auto kxrow = [&](int kq, int jq) -> T * {
        return kxr + (kq * V7_TJ + jq) * V7_W;
    };
    auto kyrow = [&](int kq, int jq) -> T * {
        return kyr + (kq * (V7_TJ + 1) + jq) * V7_W;
    };
    auto kzrow = [&](int kq, int jq) -> T * {
        return kzr + (kq * V7_TJ + jq) * V7_W;
    };
    // Element index of sweep-order column 0 of sweep-order row (j, k) in x
    // and r, in the x-faces, and in the y- and z-face arrays for the face
    // below the row; each advances by dir per column.
    auto xbase = [&](int j, int k) -> int {
        const int v = (k * ny + j) * nx;
        return BWD ? (nx * ny * nz - 1) - v : v;
    };
    auto fxbase = [&](int j, int k) -> int {
        const int jr = BWD ? ny - 1 - j : j, kr = BWD ? nz - 1 - k : k;
        return (kr * ny + jr) * (nx + 1) + (BWD ? nx : 0);
    };
    auto fybase = [&](int j, int k) -> int {
        const int jf = BWD ? ny - j : j, kr = BWD ? nz - 1 - k : k;
        return (kr * (ny + 1) + jf) * nx + (BWD ? nx - 1 : 0);
    };
    auto fzbase = [&](int j, int k) -> int {
        const int jr = BWD ? ny - 1 - j : j, kf = BWD ? nz - k : k;
        return (kf * ny + jr) * nx + (BWD ? nx - 1 : 0);
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
        for (int e = tid; e < NXR * V7_W; e += NT) xr[e] = T(0);
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0 || aborted) return;
        const int jt = tile % a.njt, vt = tile / a.njt;
        const int j0 = V7_TJ * jt, k0 = KT * vt;
        const int T0 = j0 + k0;
        const int T_start = T0 - 1 - V7_PRE;
        const int T_lastc = T0 + (V7_TJ - 1) + (KT - 1) + nx - 1;
        const int nblk = (T_lastc + 5 - T_start + 15) / 16;
        const __amdgpu_buffer_rsrc_t rs_b = __builtin_amdgcn_make_buffer_rsrc(
            a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);

        if (wv < NW) {
            // ================= compute: row (j0 + jj, k0 + kk) =============
            const int jj = l & 15, kk = 4 * wv + (l >> 4);
            const int j = j0 + jj, k = k0 + kk;
            const bool vc = j < ny && k < nz;
            const int sc = j + k;
            T *const own = xrow(kk, jj);
            const T *const yup = xrow(kk, jj + 1);
            const T *const ydn = xrow(kk, jj - 1);
            const T *const zup = xrow(kk + 1, jj);
            const T *const zdn = xrow(kk - 1, jj);
            const T *const rown = rrow(kk, jj);
            const T *const fxo = kxrow(kk, jj);
            const T *const fyo = kyrow(kk, jj);
            const T *const fyu = kyrow(kk, jj + 1);
            const T *const fzo = kzrow(kk, jj);
            const T *const fzu = kzrow(kk + 1, jj);
            const int ipub = jj == 15 ? kk : (kk == KT - 1 ? KT + jj : -1);
            const bool pub = vc && ipub >= 0;
            const int bout = (vt * a.njt + jt) * a.ns * WB + ipub - T0 * WB;
            T xprev = T(0);
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 4
                for (int ph = 0; ph < 16; ++ph) {
                    const int st = Tb + ph;
                    const int f = st - sc;
                    const int o0 = f & (V7_W - 1), o1 = (f + 1) & (V7_W - 1);
                    const T xp = own[o1], yu = yup[o0], yd = ydn[o0];
                    const T zu = zup[o0], zd = zdn[o0], rv = rown[o0];
                    const T fx0 = fxo[o0], fx1 = fxo[o1];
                    const T fy0 = fyo[o0], fy1 = fyu[o0];
                    const T fz0 = fzo[o0], fz1 = fzu[o0];
                    // real orientation: in a backward sweep the sweep-order
                    // upper neighbours and faces are the real lower ones
                    const T x =
                        BWD ? v7_combine<T>(rv, xp, xprev, yu, yd, zu, zd,
                                            fx1, fx0, fy1, fy0, fz1, fz0)
                            : v7_combine<T>(rv, xprev, xp, yd, yu, zd, zu,
                                            fx0, fx1, fy0, fy1, fz0, fz1);
                    const bool act = vc && (unsigned)f < (unsigned)nx;
                    if (act) {
                        own[o0] = x;
                        xprev = x;
                    }
                    R::store(rs_b,
                             act && pub ? (unsigned)(bout + st * WB) * RB
                                        : OOB,
                             R::make(x, ep));
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else if (wv < 2 * NW) {
            // ====== memory wavefront m: rows of compute wavefront m ======
            // At step T plane 4m + (T mod 4): lane l -> row l / 4, window
            // column l % 4.  Halo lanes: l < 8 the row j0 + 16 of that plane
            // (x, y-faces); 8 <= l < 40 of the last wavefront the plane
            // k0 + KT, rows 4 (T mod 4) .. + 3 (x, z-faces).
            const int m = wv - NW;
            const int jj = l >> 2, cq = l & 3;
            const int j = j0 + jj;
            const bool h16 = l < 8;
            const bool hpl = !h16 && m == NW - 1 && l < 40;
            const bool hx = h16 ? l < 4 : ((l - 8) >> 4) == 0;  // x or face
            const int hjoff = h16 ? 16 : ((l - 8) >> 2) & 3;
            const int nb = nx * ny * nz * (int)ES;
            const __amdgpu_buffer_rsrc_t rs_x = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.xin ? a.xin : a.r), 0, a.xin ? nb : 0, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_r = __builtin_amdgcn_make_buffer_rsrc(
                (void *)a.r, 0, nb, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_o = __builtin_amdgcn_make_buffer_rsrc(
                (void *)a.xout, 0, nb, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_fx = __builtin_amdgcn_make_buffer_rsrc(
                (void *)a.kx, 0, nz * ny * (nx + 1) * (int)ES, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_fy = __builtin_amdgcn_make_buffer_rsrc(
                (void *)a.ky, 0, nz * (ny + 1) * nx * (int)ES, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_fz = __builtin_amdgcn_make_buffer_rsrc(
                (void *)a.kz, 0, (nz + 1) * ny * nx * (int)ES, 0x00020000);
            T px[4], pr[4], pfx[4], pfy[4], pfz[4], hpx[4], hpy[4], hpz[4];
#pragma unroll
            for (int p = 0; p < 4; ++p)
                px[p] = pr[p] = pfx[p] = pfy[p] = pfz[p] = hpx[p] = hpy[p] =
                    hpz[p] = T(0);
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph0 = 0; ph0 < 16; ph0 += 4)
#pragma unroll
                for (int p4 = 0; p4 < 4; ++p4) {
                    const int st = Tb + ph0 + p4;
                    const int kk = 4 * m + p4, k = k0 + kk;
                    const bool vrow = j < ny && k < nz;
                    const int f = st - (j + k);
                    // store [f - 4, f) (read before the staging writes)
                    {
                        const int cs = f - 4 + cq;
                        const T xv = xrow(kk, jj)[cs & (V7_W - 1)];
                        buf_store<T, 0>(
                            rs_o,
                            vrow && (unsigned)cs < (unsigned)nx
                                ? (unsigned)(xbase(j, k) + dir * cs) * ES
                                : OOB,
                            xv);
                    }
                    // stage [f + 2, f + 6): write what was loaded 4 steps
                    // ago, load the window 4 columns further
                    {
                        const int c = f + 2 + cq, o = c & (V7_W - 1);
                        xrow(kk, jj)[o] = px[p4];
                        rrow(kk, jj)[o] = pr[p4];
                        kxrow(kk, jj)[o] = pfx[p4];
                        kyrow(kk, jj)[o] = pfy[p4];
                        kzrow(kk, jj)[o] = pfz[p4];
                        const int cl = c + 4;
                        const bool in = (unsigned)cl < (unsigned)nx;
                        const unsigned ox =
                            vrow && in ? (unsigned)(xbase(j, k) + dir * cl) * ES
                                       : OOB;
                        px[p4] = buf_load<T>(rs_x, ox);
                        pr[p4] = buf_load<T>(rs_r, ox);
                        pfx[p4] = buf_load<T>(
                            rs_fx, vrow && (unsigned)cl <= (unsigned)nx
                                       ? (unsigned)(fxbase(j, k) + dir * cl) *
                                             ES
                                       : OOB);
                        pfy[p4] = buf_load<T>(
                            rs_fy, j <= ny && k < nz && in
                                       ? (unsigned)(fybase(j, k) + dir * cl) *
                                             ES
                                       : OOB);
                        pfz[p4] = buf_load<T>(
                            rs_fz, j < ny && k <= nz && in
                                       ? (unsigned)(fzbase(j, k) + dir * cl) *
                                             ES
                                       : OOB);
                    }
                    // halo rows
                    {
                        const int hjj = h16 ? 16 : 4 * p4 + hjoff;
                        const int hkk = h16 ? kk : KT;
                        const int hj = j0 + hjj, hk = k0 + hkk;
                        const int c = st - (hj + hk) + 2 + cq;
                        const int o = c & (V7_W - 1);
                        if (h16 || hpl) {
                            T *const ring =
                                hx ? xrow(hkk, hjj)
                                   : (h16 ? kyrow(hkk, hjj) : kzrow(hkk, hjj));
                            ring[o] = hx ? hpx[p4] : (h16 ? hpy[p4] : hpz[p4]);
                        }
                        const int cl = c + 4;
                        const bool in = (unsigned)cl < (unsigned)nx;
                        hpx[p4] = buf_load<T>(
                            rs_x, (h16 || hpl) && hx && hj < ny && hk < nz && in
                                      ? (unsigned)(xbase(hj, hk) + dir * cl) *
                                            ES
                                      : OOB);
                        // one load per array (a buffer resource is
                        // uniform); lanes of another array read 0
                        hpy[p4] = buf_load<T>(
                            rs_fy, h16 && !hx && hj <= ny && hk < nz && in
                                       ? (unsigned)(fybase(hj, hk) + dir * cl) *
                                             ES
                                       : OOB);
                        hpz[p4] = buf_load<T>(
                            rs_fz, hpl && !hx && hj < ny && hk <= nz && in
                                       ? (unsigned)(fzbase(hj, hk) + dir * cl) *
                                             ES
                                       : OOB);
                    }
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else {
            // ====== poll wavefront: lane h < KT + 16 owns one halo row ====
            // h < KT: (jj = -1, kk = h) from tile (jt - 1, vt), entry h;
            // h = KT + jj: plane k0 - 1 row jj from (jt, vt - 1), entry
            // KT + jj (jj < 15) or KT - 1 (jj = 15)
            const int h = l;
            const bool left = h < KT;
            const int jj = left ? -1 : h - KT;
            const int kk = left ? h : -1;
            const int j = j0 + jj, k = k0 + kk;
            const int pjt = left ? jt - 1 : jt, pvt = left ? vt : vt - 1;
            const int ent = left ? h : (jj < 15 ? KT + jj : KT - 1);
            const bool hv = h < NH && j >= 0 && j < ny && k >= 0 && k < nz;
            const int hs = j + k;
            const int hT0 = V7_TJ * pjt + KT * pvt;
            const int hslot =
                hv ? (pvt * a.njt + pjt) * a.ns * WB + ent : 0;
            T *const hrow = xrow(hv ? kk : 0, hv ? jj : 0);
            auto pslice = [&](int T_) -> int {
                const int s = min(max(T_ - hT0, 0), a.ns - 1);
                return hslot + s * WB;
            };
            typename R::V ppipe[POLL];
#pragma unroll
            for (int p = 0; p < POLL; ++p) ppipe[p] = typename R::V{};
            int spin_budget = a.spin_limit;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph0 = 0; ph0 < 16; ph0 += 4)
#pragma unroll
                for (int ph = 0; ph < 4; ++ph) {
                    const int st = Tb + ph0 + ph;
                    const int c = st - hs;
                    if (hv && c >= 0) {
                        T v = T(0);
                        if (c < nx) {
                            typename R::V rec = ppipe[ph & (POLL - 1)];
                            const unsigned src = (unsigned)pslice(st) * RB;
                            bool retried = false;
                            while (!R::ready(rec, ep)) {
                                retried = true;
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
                                rec = R::load(rs_b, src);
                            }
                            v = R::value(rec);
                            // caught up: the slices preloaded before the
                            // wait were loaded too early too; load them again
                            if (retried) {
#pragma unroll
                                for (int q = 1; q < POLL; ++q)
                                    ppipe[(ph + q) & (POLL - 1)] = R::load(
                                        rs_b, (unsigned)pslice(st + q) * RB);
                            }
                        }
                        hrow[c & (V7_W - 1)] = v;
                    }
                    ppipe[ph & (POLL - 1)] = R::load(
                        rs_b,
                        hv ? (unsigned)pslice(st + POLL) * RB : OOB);
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

V7Layout v7_layout(Grid g, int nw)
{
    V7Layout L{};
    L.nw = nw;
    L.kt = 4 * nw;
    L.njt = (g.ny + V7_TJ - 1) / V7_TJ;
    L.nbands = (g.nz + L.kt - 1) / L.kt;
    L.ntiles = L.njt * L.nbands;
    L.ns = g.nx + (V7_TJ - 1) + (L.kt - 1);
    L.wb = L.kt + 15;
    L.bnd_elems = (int64_t)L.ntiles * L.ns * L.wb;
    return L;
}

size_t v7_lds_bytes(int nw, m2s_dtype t)
{
    const size_t kt = 4 * (size_t)nw;
    const size_t rows = (kt + 2) * V7_RJ + 2 * kt * V7_TJ +
                        kt * (V7_TJ + 1) + (kt + 1) * V7_TJ;
    return rows * V7_W * (t == M2S_F64 ? 8 : 4);
}

int v7_threads(int nw) { return 64 * (2 * nw + 1); }

template <typename T, bool BWD, int NW, int POLL>
static hipError_t v7_launch_tp(const V7Args<T> &a, int grid, size_t lds,
                              hipStream_t s)
{
    auto k = v7_tile_kernel<T, BWD, NW, POLL>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
            160 * 1024 - 64);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * (2 * NW + 1)), lds, s, a);
    return hipGetLastError();
}

template <typename T, bool BWD, int NW>
static hipError_t v7_launch_t(const V7Args<T> &a, int grid, size_t lds,
                              hipStream_t s)
{
    return v7_poll(a.ntiles, grid) == 2
               ? v7_launch_tp<T, BWD, NW, 2>(a, grid, lds, s)
               : v7_launch_tp<T, BWD, NW, 4>(a, grid, lds, s);
}

template <typename T>
static hipError_t v7_launch_typed(const m2s_stencil &A, const void *r,
                                  const void *xin, void *xout, bool bwd,
                                  Workspace &ws, const SweepPlan &plan,
                                  hipStream_t s)
{
    const int nw = plan.slab_planes / 4;
    const size_t lds = v7_lds_bytes(nw, A.dtype);
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    if (++ws.epoch == 0) ++ws.epoch;
    V7Args<T> a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.ntiles = plan.nslabs;
    a.njt = ws.tile_nutb;
    a.ns = ws.tile_ns;
    a.r = (const T *)r;
    a.xin = (const T *)xin;
    a.xout = (T *)xout;
    a.kx = (const T *)A.kx;
    a.ky = (const T *)A.ky;
    a.kz = (const T *)A.kz;
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = ws.epoch;
    a.ticket = ws.ticket;
    a.ticket_base = base;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    switch (nw) {
    case 1:
        return bwd ? v7_launch_t<T, true, 1>(a, plan.grid, lds, s)
                   : v7_launch_t<T, false, 1>(a, plan.grid, lds, s);
    case 2:
        return bwd ? v7_launch_t<T, true, 2>(a, plan.grid, lds, s)
                   : v7_launch_t<T, false, 2>(a, plan.grid, lds, s);
    case 4:
        return bwd ? v7_launch_t<T, true, 4>(a, plan.grid, lds, s)
                   : v7_launch_t<T, false, 4>(a, plan.grid, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep7v(const m2s_stencil &A, const void *r,
                          const void *xin, void *xout, bool bwd,
                          Workspace &ws, const SweepPlan &plan, hipStream_t s)
{
    return A.dtype == M2S_F64
               ? v7_launch_typed<double>(A, r, xin, xout, bwd, ws, plan, s)
               : v7_launch_typed<float>(A, r, xin, xout, bwd, ws, plan, s);
}

}  // namespace m2s
