// k_sweep27.hip -- the exact lexicographic Gauss-Seidel half-sweep of the
// 27-point operator (the HPCG SymGS of Sec. 7.1; a Seidel-style stencil,
// Sec. 2.1.2) as a persistent, tiled wavefront kernel for gfx950.
//
// Schedule.  Point (i, j, k) runs at global step T = i + 2j + 4k, the
// hyperplane of Eq. (hyperplane) with weights (1, 2, 4) (Sec. 6.1.3): every
// lower neighbour has a strictly smaller T, and no two points of one step
// depend on each other.  Rows (j, k) are addressed by (u, k) with u = j + k,
// so that T = i + 2u + 2k.  A tile is 16 consecutive u by KT = 4 * NW
// consecutive k (NW wavefronts, one lane per row); the lower neighbours of
// its rows lie in the tile itself or in tiles (u - 1, k), (u, k - 1) and
// (u - 1, k - 1) of the tile grid, so the tile graph is acyclic (plain (j, k)
// boxes are not: (j + 1, k - 1) is a lower neighbour of (j, k)).  Tiles are
// handed out from a ticket counter in lexicographic (k-tile, u-tile) order,
// so a tile only ever waits for one that a running workgroup owns.
//
// Data path inside a tile (one workgroup barrier per step).
//  * LDS "current x" rings, 32 columns per row, for the tile's rows plus the
//    halo rows u0 - 2 .. u0 + 17 and planes k0 - 1 .. k0 + KT: a slot holds
//    the old value of its column until the owner updates it and the new one
//    afterwards -- the in-place semantics of the Seidel loop, kept only for
//    the columns around each row's front.  Lanes of a row group sit at
//    different columns (skew 2 per u); the padded stride 33 keeps the skewed
//    64-bit reads bank-conflict free.
//  * Coalesced HBM access: every 16 steps each row's next 16 columns of
//    x_in and r are read by 16 lanes at once (4 rows per wavefront load; one
//    group of rows per phase of the 16-step cycle), parked one cycle in
//    registers, then written into the rings; finished 16-column pieces of
//    x_out leave the ring the same way.  Buffer loads return 0 outside a row
//    or the grid, which is exactly the Dirichlet padding the rings need.
//  * A point needs the 8 neighbour rows of column i + 1.  Six of them and
//    the row's own old value are read one step early (with the column sum
//    of column i and the combination B of the point); only v2 + v3, the two
//    values written in the previous step, are read on the critical path.
//    The association is that of the sequential kernel (c27_col in
//    k_sweep.hip, c27_combine), so the two agree bit for bit.
//  * Between tiles, the new values of the rows that neighbour tiles read
//    (u0 + 14, u0 + 15 of every plane, u0 .. u0 + 13 of the top plane) go to
//    a per-tile boundary store laid out by step: slice T holds every
//    boundary row's value of step T contiguously, so producer and consumer
//    each touch one or two cache lines per step.  Each value is written once
//    as a record tagged with the launch's epoch; consumers poll the records
//    themselves (one memory round trip, no fences, no resets: any number of
//    tiles may read a record) and write the value into their rings one step
//    before its first use.
//  * Every memory instruction of a step is issued unconditionally (inactive
//    lanes use an out-of-range buffer offset, which reads 0 and drops
//    stores), so the number of instructions in flight is the same on every
//    path and the waits the compiler places cover the whole prefetch
//    distance.
#include "m2s_internal.hpp"
#include "tile_common.hpp"

#include <algorithm>
#include <cstdlib>
#include <vector>

namespace m2s {

constexpr int C27_TU = 16;    // u-rows per tile
constexpr int C27_RU = 20;    // ring rows per plane: uu = -2 .. 17
constexpr int C27_W = 32;     // x-ring columns
constexpr int C27_WP = 33;    // padded x-ring stride
constexpr int C27_WR = 16;    // r-ring columns
constexpr int C27_WRP = 17;   // padded r-ring stride
// Boundary poll distance (steps).  The poll wavefront loads the record of
// step T + C27_POLL at step T, into a ring of C27_PRING registers.  A
// consumer tile settles at a lag of about the distance plus one
// device-scope round trip behind its neighbour, and every tile crossing on
// the critical path pays that lag; a shorter distance cuts it but lets a
// record that arrives late stall the consumer a whole round trip.  3 steps
// in a ring of 4 measured best overall (1 to 4 tried, with rings of 1, 2, 4).
constexpr int C27_POLL = 3;
constexpr int C27_PRING = 4;  // a power of 2 dividing the 16-step block
static_assert(C27_POLL <= C27_PRING && 16 % C27_PRING == 0,
              "a polled slot is checked before it is reloaded");
constexpr int C27_PRE = 18;   // steps before the smallest row skew

template <typename T>
struct C27Args {
    Grid g;
    int ntiles;          // tiles, in ticket order
    int nutb;            // boundary-store tile slots per k-tile
    int ns;              // boundary slices per tile
    const int2 *tiles;   // (u-tile, k-tile) per ticket
    const T *r;
    const T *xin;        // nullptr: start from zero
    T *xout;
    double *xwide;       // WIDE: the FP32 sweep's output, widened to FP64
    T off, inv_diag;
    // ILU modes (see the kernel): per-point weight w = 1 / d, and the
    // constant diagonal of the factor sweep
    const T *w;
    T diagc;
    void *bnd;           // boundary store (records)
    int64_t bnd_elems;   // records
    unsigned epoch;      // this launch's tag, never 0
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

// Boundary-store slot of tile (ut, vt); the u-tiles of k-tile vt start at
// floor(k0 / 16).
__host__ __device__ inline int c27_slot(int ut, int vt, int KT, int nutb)
{
    return vt * nutb + (ut - (KT * vt) / C27_TU);
}

// Wavefront roles.  NW compute wavefronts (one lane per row: LDS rings and
// FP64 only, plus the device-scope boundary publication, which nothing waits
// on); NW memory wavefronts (memory wavefront m stages the old values and r
// of compute wavefront m's rows and stores its finished pieces); one poll
// wavefront (the boundary records of the neighbour tiles).  Each role runs
// its own step loop with the same number of barriers, so every wavefront
// waits only for its own memory instructions.  A value written in step T by
// one wavefront is first read in step T + 1 by another.
// MODE selects what a point computes from S, the sum over its 13 lower
// neighbours in sweep order (ZERO: the upper ones are 0 then):
//   0  SymGS      x = (r - off (S + upper)) / diag
//   1  ILU factor w = 1 / (diagc - off S)        (off = off^2, x is w)
//   2  ILU lower  y = (r - off S) w
//   3  ILU upper  z = r - off S w                (backward sweep, r = y)
// WIDE (FP32 SymGS only): the finished values are stored widened to FP64
// into xwide instead of xout -- the last sweep of a mixed-precision V-cycle
// hands its result to the FP64 solver without a conversion pass.
template <typename T, bool BWD, bool ZERO, int NW, int MODE, bool WIDE = false>
__global__ void __launch_bounds__(64 * (2 * NW + 1))
    c27_tile_kernel(C27Args<T> a)
{
    constexpr int KT = 4 * NW;           // planes per tile
    constexpr int WB = 2 * KT + 14;      // boundary slice width (records)
    constexpr int NRING = (KT + 2) * C27_RU;
    constexpr int PS = C27_RU * C27_WP;  // ring plane stride
    constexpr int RW = C27_WP;           // ring row stride
    constexpr int NT = 64 * (2 * NW + 1);
    constexpr unsigned TS = sizeof(T);
    extern __shared__ unsigned char smem_raw[];
    T *const xr = (T *)smem_raw;
    T *const rr = xr + NRING * C27_WP;
    T *const wr = rr + KT * C27_TU * C27_WRP;  // ILU modes 2, 3
    __shared__ int s_tile, s_abort;

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int last = (int)a.g.size() - 1;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int sub = l >> 4, cl = l & 15;
    const int dir = BWD ? -1 : 1;
    const unsigned OOB = 0x80000000u;    // reads 0, drops stores
    const T zero = T(0);
    const T off = a.off, inv_diag = a.inv_diag;
    const int nbytes = (int)((unsigned)(last + 1) * TS);
    using R = Rec<T>;
    constexpr unsigned RB = R::bytes;
    const unsigned ep = a.epoch;

    auto xrow = [&](int kq, int uq) -> T * {
        return xr + ((kq + 1) * C27_RU + (uq + 2)) * C27_WP;
    };
    auto rrow = [&](int kq, int uq) -> T * {
        return rr + (kq * C27_TU + uq) * C27_WRP;
    };
    auto wrow = [&](int kq, int uq) -> T * {
        return wr + (kq * C27_TU + uq) * C27_WRP;
    };
    // element index of virtual column 0 of row (j, k); dir steps along it
    auto rowbase = [&](int j, int k) -> int {
        const int v = (k * ny + j) * nx;
        return BWD ? last - v : v;
    };
    // byte offset of column c of a row; OOB outside the row or the grid
    auto boff = [&](bool vrow, int rb, int c) -> unsigned {
        return (vrow && (unsigned)c < (unsigned)nx)
                   ? (unsigned)(rb + dir * c) * TS
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
        for (int e = tid; e < NRING * C27_WP; e += NT) xr[e] = zero;
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0 || aborted) return;
        const int2 tv = a.tiles[tile];
        const int ut = tv.x, vt = tv.y;
        const int u0 = C27_TU * ut, k0 = KT * vt;
        const int T0 = 2 * (u0 + k0);  // step of column 0 of row (u0, k0)
        // step range: the first window holding column 0 of the lowest row
        // (skew T0) is loaded 16 to 23 steps before that column, the first
        // halo poll (skew T0 - 6) 8 steps before; the last row's last piece
        // is stored within 8 steps after its last column
        const int T_start = T0 - 6 - C27_PRE;
        const int T_lastc = T0 + 2 * (C27_TU - 1) + 2 * (KT - 1) + nx - 1;
        const int nblk = (T_lastc + 9 - T_start + 15) / 16;

        if (wv < NW) {
            // ================= compute: row (u0 + cl, k0 + kk) =============
            const int kk = 4 * wv + sub;
            const int uc = u0 + cl, kc = k0 + kk, jc = uc - kc;
            const bool vc = (unsigned)jc < (unsigned)ny && kc < nz;
            const int sc = 2 * (uc + kc);
            T *const own = xrow(kk, cl);
            T *const rown = rrow(kk, cl);
            T *const wown = wrow(kk, cl);
            // boundary rows: u0 + 14, u0 + 15 of every plane (entries 0 ..
            // 2KT - 1) and u0 .. u0 + 13 of the top plane (2KT .. 2KT + 13)
            const int ipub = cl >= 14 ? (cl - 14) + 2 * kk
                                      : (kk == KT - 1 ? 2 * KT + cl : -1);
            const bool pub = vc && ipub >= 0;
            const int bout =
                c27_slot(ut, vt, KT, a.nutb) * a.ns * WB + ipub - T0 * WB;
            const __amdgpu_buffer_rsrc_t rs_b =
                __builtin_amdgcn_make_buffer_rsrc(
                    a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);
            // carried between steps: F(f) = A(f) + D(f) (F0), A(f + 1) (An)
            // and B of the next point (Bn); only D(f + 1) = v2 + v3, the
            // two values written in the previous step, is read on the
            // critical path
            T F0 = zero, An = zero, Bn = zero, xprev = zero;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll
                for (int ph = 0; ph < 16; ++ph) {
                    const int st = Tb + ph;
                    const int f = st - sc;
                    const int c1 = (f + 1) & (C27_W - 1);
                    const int c2 = (f + 2) & (C27_W - 1);
                    const T v2 = own[c1 - PS], v3 = own[c1 - RW];
                    const T v0 = own[c2 - PS - 2 * RW], v1 = own[c2 - PS - RW];
                    const T v4 = own[c2 + RW], v5 = own[c2 + PS];
                    const T v6 = own[c2 + PS + RW];
                    const T v7 = own[c2 + PS + 2 * RW];
                    const T xo2 = own[c2];
                    const T rf = MODE == 1 ? a.diagc : rown[f & (C27_WR - 1)];
                    const T D = v2 + v3;
                    T x;
                    if constexpr (MODE == 0) {
                        x = c27_combine(rf, Bn, D, xprev, off, inv_diag);
                    } else if constexpr (MODE == 1) {
                        x = T(1) / c27_combine(rf, Bn, D, xprev, off, T(1));
                    } else if constexpr (MODE == 2) {
                        x = c27_combine(rf, Bn, D, xprev, off,
                                        wown[f & (C27_WR - 1)]);
                    } else {
                        const T t = c27_combine(zero, Bn, D, xprev, off, T(1));
                        x = fma(t, wown[f & (C27_WR - 1)], rf);
                    }
                    const bool act = vc && (unsigned)f < (unsigned)nx;
                    if (act) {
                        own[f & (C27_W - 1)] = x;
                        xprev = x;
                    }
                    R::store(rs_b,
                             act && pub ? (unsigned)(bout + st * WB) * RB : OOB,
                             R::make(x, ep));
                    const T Fp = An + D;  // F(f + 1)
                    An = ((v0 + v1) + (v4 + v5)) + (v6 + v7);  // A(f + 2)
                    Bn = (F0 + Fp) + (An + xo2);
                    F0 = Fp;
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else if (wv < 2 * NW) {
            // ====== memory wavefront m: rows of compute wavefront m ======
            const int m = wv - NW;
            const __amdgpu_buffer_rsrc_t rs_r =
                __builtin_amdgcn_make_buffer_rsrc((void *)a.r, 0, nbytes,
                                                  0x00020000);
            const __amdgpu_buffer_rsrc_t rs_x =
                __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(ZERO ? a.r : a.xin), 0, nbytes, 0x00020000);
            static_assert(!WIDE || (sizeof(T) == 4 && MODE == 0),
                          "widened output is for the FP32 SymGS sweep");
            const __amdgpu_buffer_rsrc_t rs_o =
                WIDE ? __builtin_amdgcn_make_buffer_rsrc(
                           (void *)a.xwide, 0,
                           (int)((unsigned)(last + 1) * 8u), 0x00020000)
                     : __builtin_amdgcn_make_buffer_rsrc((void *)a.xout, 0,
                                                         nbytes, 0x00020000);
            const __amdgpu_buffer_rsrc_t rs_w =
                __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(MODE >= 2 ? a.w : a.xout), 0,
                    MODE >= 2 ? nbytes : 0, 0x00020000);
            // Rows of step T: rho = 8 (T mod 8) + lane / 8, column lane % 8;
            // each row gets an 8-column window of x_old ([f + 9, f + 17)),
            // of r ([f + 1, f + 9)) and stores its finished [f - 8, f)
            // every 8 steps; loads are parked 8 steps in registers.
            T xpipe[8], rpipe[8], hpipe[8], wpipe[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                xpipe[q] = rpipe[q] = hpipe[q] = wpipe[q] = zero;
            const int q8 = l & 7, r8 = l >> 3;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll
                for (int ph = 0; ph < 16; ++ph) {
                    const int st = Tb + ph;
                    const int p8 = ph & 7;
                    {
                        const int rho = 8 * p8 + r8;
                        const int uL = rho & 15, kL = 4 * m + (rho >> 4);
                        const int u = u0 + uL, k = k0 + kL, j = u - k;
                        const bool v = (unsigned)j < (unsigned)ny && k < nz;
                        const int f = st - 2 * (u + k);
                        const int rb = v ? rowbase(j, k) : 0;
                        T *const xw = xrow(kL, uL);
                        const int cx = f + 9 + q8, cr = f + 1 + q8,
                                  cs = f - 8 + q8;
                        xw[cx & (C27_W - 1)] = xpipe[p8];
                        rrow(kL, uL)[cr & (C27_WR - 1)] = rpipe[p8];
                        if constexpr (MODE >= 2)
                            wrow(kL, uL)[cr & (C27_WR - 1)] = wpipe[p8];
                        const T xv = xw[cs & (C27_W - 1)];
                        if (!ZERO)
                            xpipe[p8] = buf_load<T>(rs_x, boff(v, rb, cx + 8));
                        if constexpr (MODE != 1)
                            rpipe[p8] = buf_load<T>(rs_r, boff(v, rb, cr + 8));
                        if constexpr (MODE >= 2)
                            wpipe[p8] = buf_load<T>(rs_w, boff(v, rb, cr + 8));
                        if constexpr (WIDE)
                            buf_store<double, 0>(
                                rs_o,
                                (v && (unsigned)cs < (unsigned)nx)
                                    ? (unsigned)(rb + dir * cs) * 8u
                                    : OOB,
                                (double)xv);
                        else
                            buf_store<T, 0>(rs_o, boff(v, rb, cs), xv);
                    }
                    // -- old-value halo rows: u0 + 16, u0 + 17 of this
                    //    wavefront's planes (h < 8) and plane k0 + KT
                    //    (h = 8 .. 25, last wavefront), 8 rows per step --
                    if (p8 < 4) {
                        const int h = 8 * p8 + r8;
                        const bool lo = h < 8;
                        const bool mine = lo || (m == NW - 1 && h < 26);
                        const int uH = lo ? 16 + (h & 1) : h - 8;
                        const int kH = lo ? 4 * m + (h >> 1) : KT;
                        const int u = u0 + uH, k = k0 + kH, j = u - k;
                        const bool v = mine && (unsigned)j < (unsigned)ny &&
                                       k < nz;
                        const int cx = st - 2 * (u + k) + 9 + q8;
                        if (mine) xrow(kH, uH)[cx & (C27_W - 1)] = hpipe[p8];
                        const int rb = v ? rowbase(j, k) : 0;
                        if (!ZERO)
                            hpipe[p8] = buf_load<T>(rs_x, boff(v, rb, cx + 8));
                    }
                    __syncthreads();
                }
                if (s_abort) {
                    aborted = true;
                    break;
                }
            }
        } else {
            // ====== poll wavefront: lane h < 2KT + 18 owns one new-value
            //        halo row and the tile / entry that publishes it ======
            int hu = 0, hk = 0, hidx = 0, put = ut, pvt = vt;
            if (l < 2 * KT) {  // u0 - 2, u0 - 1 of plane k0 + l / 2
                hu = -2 + (l & 1); hk = l >> 1; hidx = l; put = ut - 1;
            } else if (l < 2 * KT + 14) {  // plane k0 - 1, u0 .. u0 + 13
                hu = l - 2 * KT; hk = -1; hidx = 2 * KT + hu; pvt = vt - 1;
            } else if (l < 2 * KT + 16) {  // plane k0 - 1, u0 + 14, u0 + 15
                hu = 14 + (l - 2 * KT - 14); hk = -1;
                hidx = 2 * (KT - 1) + (hu - 14); pvt = vt - 1;
            } else if (l < 2 * KT + 18) {  // plane k0 - 1, u0 - 2, u0 - 1
                hu = -2 + (l - 2 * KT - 16); hk = -1;
                hidx = 2 * (KT - 1) + (hu + 2); put = ut - 1; pvt = vt - 1;
            }
            const int hug = u0 + hu, hkg = k0 + hk, hj = hug - hkg;
            const bool vh = l < 2 * KT + 18 && (unsigned)hj < (unsigned)ny &&
                            hkg >= 0 && hkg < nz;
            const int sh = 2 * (hug + hkg);
            const int T0p = 2 * (C27_TU * put + KT * pvt);
            const int pbuf =
                vh ? c27_slot(put, pvt, KT, a.nutb) * a.ns * WB + hidx : 0;
            T *const hrow = xrow(vh ? hk : 0, vh ? hu : 0);
            const __amdgpu_buffer_rsrc_t rs_b =
                __builtin_amdgcn_make_buffer_rsrc(
                    a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);
            // record index of this lane's entry in slice T_
            auto pslice = [&](int T_) -> int {
                const int q = min(max(T_ - T0p, 0), a.ns - 1);
                return pbuf + q * WB;
            };
            typename R::V ppipe[C27_PRING];
#pragma unroll
            for (int q = 0; q < C27_PRING; ++q) ppipe[q] = typename R::V{};
            int spin_budget = a.spin_limit;
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll
                for (int ph = 0; ph < 16; ++ph) {
                    const int st = Tb + ph;
                    const int c = st - sh;
                    if (vh && c >= 0) {
                        T v = zero;
                        if (c < nx) {
                            typename R::V rec = ppipe[ph & (C27_PRING - 1)];
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
                            // a record that had to be waited for means the
                            // consumer has caught up: the slices preloaded
                            // before the wait were loaded too early as well,
                            // so load them again (256^3: 553 -> 537 us)
                            if (retried) {
#pragma unroll
                                for (int q = 1; q < C27_POLL; ++q)
                                    ppipe[(ph + q) & (C27_PRING - 1)] = R::load(
                                        rs_b, (unsigned)pslice(st + q) * RB);
                            }
                        }
                        hrow[c & (C27_W - 1)] = v;
                    }
                    // poll the slice C27_POLL steps ahead; its ring slot was
                    // checked C27_PRING - C27_POLL steps ago
                    ppipe[(ph + C27_POLL) & (C27_PRING - 1)] = R::load(
                        rs_b, vh ? (unsigned)pslice(st + C27_POLL) * RB : OOB);
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

C27Layout c27_layout(Grid g, int nw)
{
    C27Layout L{};
    L.nw = nw;
    L.kt = 4 * nw;
    L.nbands = (g.nz + L.kt - 1) / L.kt;
    L.ns = g.nx + 2 * (C27_TU - 1) + 2 * (L.kt - 1);
    L.wb = 2 * L.kt + 14;
    L.nutb = 0;
    for (int vt = 0; vt < L.nbands; ++vt) {
        const int k0 = L.kt * vt, kmax = std::min(k0 + L.kt, g.nz) - 1;
        const int utmin = k0 / C27_TU, utmax = (kmax + g.ny - 1) / C27_TU;
        L.nutb = std::max(L.nutb, utmax - utmin + 1);
        for (int ut = utmin; ut <= utmax; ++ut) {
            // the tile holds a row (u, k) with 0 <= u - k < ny
            const int ulo = C27_TU * ut, uhi = ulo + C27_TU - 1;
            const int klo = std::max(k0, ulo - g.ny + 1);
            const int khi = std::min(kmax, uhi);
            if (klo <= khi) L.tiles.push_back(int2{ut, vt});
        }
    }
    L.bnd_elems = (int64_t)L.nbands * L.nutb * L.ns * L.wb;
    return L;
}

int c27_threads(int nw) { return 64 * (2 * nw + 1); }

size_t c27_lds_bytes(int nw, m2s_dtype t, int mode)
{
    const int kt = 4 * nw;
    const size_t es = t == M2S_F64 ? 8 : 4;
    return ((size_t)(kt + 2) * C27_RU * C27_WP +
            (size_t)(mode >= 2 ? 2 : 1) * kt * C27_TU * C27_WRP) *
           es;
}

template <typename T, bool BWD, bool ZERO, int NW, int MODE = 0,
          bool WIDE = false>
static hipError_t c27_launch_t(const C27Args<T> &a, int grid, size_t lds,
                               hipStream_t s)
{
    auto k = c27_tile_kernel<T, BWD, ZERO, NW, MODE, WIDE>;
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

template <typename T, bool BWD, bool ZERO>
static hipError_t c27_launch_nw(const C27Args<T> &a, int nw, int grid,
                                size_t lds, hipStream_t s)
{
    switch (nw) {
    case 1: return c27_launch_t<T, BWD, ZERO, 1>(a, grid, lds, s);
    case 2: return c27_launch_t<T, BWD, ZERO, 2>(a, grid, lds, s);
    case 4: return c27_launch_t<T, BWD, ZERO, 4>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t c27_launch_dir(const C27Args<T> &a, bool bwd, bool zero,
                                 int nw, int grid, size_t lds, hipStream_t s)
{
    if (bwd)
        return zero ? c27_launch_nw<T, true, true>(a, nw, grid, lds, s)
                    : c27_launch_nw<T, true, false>(a, nw, grid, lds, s);
    return zero ? c27_launch_nw<T, false, true>(a, nw, grid, lds, s)
                : c27_launch_nw<T, false, false>(a, nw, grid, lds, s);
}

template <int MODE, bool BWD>
static hipError_t c27_launch_dilu(const C27Args<double> &a, int nw, int grid,
                                 size_t lds, hipStream_t s)
{
    // 4 compute wavefronts would need more LDS than a CU has with the
    // weight ring
    switch (nw) {
    case 1: return c27_launch_t<double, BWD, true, 1, MODE>(a, grid, lds, s);
    case 2: return c27_launch_t<double, BWD, true, 2, MODE>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dilu27(const m2s_stencil &A, int mode, const void *r,
                        const void *w, void *out, Workspace &ws,
                        const SweepPlan &plan, hipStream_t s)
{
    const int nw = plan.slab_planes / 4;
    // reject before the workspace's ticket base and epoch move
    if (A.dtype != M2S_F64 || (nw != 1 && nw != 2) || mode < 1 || mode > 3)
        return hipErrorInvalidValue;
    const size_t lds = c27_lds_bytes(nw, A.dtype, mode);
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    if (++ws.epoch == 0) ++ws.epoch;
    C27Args<double> a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.ntiles = plan.nslabs;
    a.nutb = ws.tile_nutb;
    a.ns = ws.tile_ns;
    a.tiles = ws.tile_list;
    a.ticket = ws.ticket;
    a.ticket_base = base;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    a.r = (const double *)(r ? r : out);
    a.xin = nullptr;
    a.xout = (double *)out;
    a.w = (const double *)w;
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = ws.epoch;
    switch (mode) {
    case 1:  // factor: w = 1 / (diag - off^2 S), forward
        a.off = A.offdiag * A.offdiag;
        a.diagc = A.diag;
        return c27_launch_dilu<1, false>(a, nw, plan.grid, lds, s);
    case 2:  // lower solve, forward
        a.off = A.offdiag;
        return c27_launch_dilu<2, false>(a, nw, plan.grid, lds, s);
    case 3:  // upper solve, backward
        a.off = A.offdiag;
        return c27_launch_dilu<3, true>(a, nw, plan.grid, lds, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep27(const m2s_stencil &A, const void *r,
                          const void *xin, void *xout, bool bwd,
                          Workspace &ws, const SweepPlan &plan, hipStream_t s)
{
    const int nw = plan.slab_planes / 4;
    const size_t lds = c27_lds_bytes(nw, A.dtype, 0);
    // this launch takes tickets [base, base + ntiles + grid)
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    // boundary records of earlier launches carry other epochs
    if (++ws.epoch == 0) ++ws.epoch;
    const unsigned epoch = ws.epoch;
    auto fill = [&](auto &a) {
        a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
        a.ntiles = plan.nslabs;
        a.nutb = ws.tile_nutb;
        a.ns = ws.tile_ns;
        a.tiles = ws.tile_list;
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
        a.bnd = ws.bnd;
        a.bnd_elems = ws.bnd_elems;
        a.epoch = epoch;
        return c27_launch_dir(a, bwd, zero, nw, plan.grid, lds, s);
    }
    C27Args<float> a{};
    fill(a);
    a.r = (const float *)r;
    a.xin = (const float *)xin;
    a.xout = (float *)xout;
    a.off = (float)A.offdiag;
    a.inv_diag = (float)(1.0 / A.diag);
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = epoch;
    return c27_launch_dir(a, bwd, zero, nw, plan.grid, lds, s);
}

hipError_t launch_sweep27_wide(const m2s_stencil &A, const void *r,
                               const void *xin, double *xout, Workspace &ws,
                               const SweepPlan &plan, hipStream_t s)
{
    const int nw = plan.slab_planes / 4;
    // the widened output is addressed with 32-bit byte offsets too
    const int64_t n = (int64_t)A.ext.nx * A.ext.ny * A.ext.nz;
    if (A.dtype != M2S_F32 || !xin || n * 8 >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    const size_t lds = c27_lds_bytes(nw, A.dtype, 0);
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    if (++ws.epoch == 0) ++ws.epoch;
    C27Args<float> a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.ntiles = plan.nslabs;
    a.nutb = ws.tile_nutb;
    a.ns = ws.tile_ns;
    a.tiles = ws.tile_list;
    a.ticket = ws.ticket;
    a.ticket_base = base;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    a.r = (const float *)r;
    a.xin = (const float *)xin;
    a.xout = nullptr;
    a.xwide = xout;
    a.off = (float)A.offdiag;
    a.inv_diag = (float)(1.0 / A.diag);
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = ws.epoch;
    switch (nw) {
    case 1: return c27_launch_t<float, true, false, 1, 0, true>(a, plan.grid, lds, s);
    case 2: return c27_launch_t<float, true, false, 2, 0, true>(a, plan.grid, lds, s);
    case 4: return c27_launch_t<float, true, false, 4, 0, true>(a, plan.grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace m2s
