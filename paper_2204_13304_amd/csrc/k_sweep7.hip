// k_sweep7.hip -- the block SSOR half-sweep of the NPB-LU-shaped BLOCK7x5
// operator (7-point stencil, 5 unknowns per point, constant 5x5 blocks;
// Sec. 7.1) as a persistent, tiled wavefront kernel for gfx950.
//
// Schedule.  Point (i, j, k) runs at step T = i + j + k, the hyperplane of
// Eq. (hyperplane) with unit weights (Sec. 6.1.3): the three lower
// neighbours have smaller T.  A tile is 16 consecutive j by 4 consecutive
// k, one lane per row; the lower neighbours of its rows lie in the tile or
// in tiles (j - 1, k) and (j, k - 1) of the tile grid (rectangular tiles
// are acyclic for 7 points).  Tiles are handed out from a ticket counter in
// the order of their first step j0 + k0.
//
// The point update is split into b7_upper / b7_relax / b7_lower, so that
// only its last part -- the three lower neighbours' new values times
// w D^{-1} B_d -- lies on the step-to-step critical path; the parts that
// need only old values run ahead of the front in wavefronts of their own.
// Each wavefront keeps the coefficients of its part in registers.  Roles
// (b7_role maps them to wavefronts):
//   0 compute   x(f) = g(f) - sum_lower W_d x_d at the row's front f
//   1 upper     u(f + 2) = b - sum_upper B_d x_d (old values: the upper
//               neighbours reach column f + 2 only after this step)
//   2 relax     g(f + 1) = (1 - w) x_old(f + 1) + G u(f + 1)
//   3 x memory  stages x_old windows [f + 4, f + 8) (loads are parked in
//               registers for 8 steps, two services of the plane, to cover
//               the memory latency)
//   4 poll      the neighbour tiles' boundary records (new values)
//   5 b memory  stages b windows [f + 3, f + 7) and the old values of the
//               halo rows (row 16 of every plane, plane 4)
//   6 x stores  stores the finished columns [f - 4, f)
// The memory wavefronts serve the 4 planes in turn, one per step, with
// 4-column windows (element l + 64q -> row (l + 64q) / 20, column
// ((l + 64q) % 20) / 5, component (l + 64q) % 5).  Every role runs the same
// barriers; a value written by one wavefront in step T is read by another
// from step T + 1 on.  Boundary rows (j0 + 15 of every plane, j0 .. j0 + 14
// of the top plane) publish one epoch-tagged record per component and
// step, laid out component-major within a step's slice, so that a store or
// poll instruction touches consecutive records; consumers poll them one
// step ahead.
#include "m2s_internal.hpp"
#include "tile_common.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace m2s {

constexpr int B7_TJ = 16;    // j-rows per tile
constexpr int B7_KT = 4;     // planes per tile
constexpr int B7_RJ = 18;    // x-ring rows per plane: jj = -1 .. 16
constexpr int B7_W = 16;     // x-ring columns
// Ring row strides (doubles).  The rows' column skew spreads a step's
// accesses over the banks by itself, so the x and b rings are unpadded (a
// padding of one double put four lanes of a 16-lane pass of a 64-bit access
// on one pair of banks); the 4-column u and g rings are padded by 2
// (unpadded: four lanes on one pair, now two).
constexpr int B7_RS = 80;    // x ring: 16 columns x 5
constexpr int B7_BS = 40;    // b ring: 8 columns x 5
constexpr int B7_US = 22;    // u and g rings: 4 columns x 5, + 2
// Boundary poll distance (steps) and the ring of registers the polled
// records wait in.  A consumer settles about POLL steps plus a record round
// trip behind its neighbour, and the poll wavefront waits, every step, for
// the record it loaded POLL steps earlier.
constexpr int B7_POLL = 1;
constexpr int B7_PRING = 1;  // a power of 2 dividing the 4-step unroll
static_assert(B7_POLL <= B7_PRING && 4 % B7_PRING == 0,
              "a polled slot is checked before it is reloaded");
constexpr int B7_PRE = 20;   // steps before the smallest row skew
constexpr int B7_NT = 448;   // seven wavefronts
// Role of wavefront w.  Wavefronts w and w + 4 share a SIMD: upper, which
// issues the most instructions per step, gets a SIMD of its own, compute
// shares one with the x stores (measured 1 % faster than the other way
// round), and the other light roles go in pairs (b memory + poll, x memory
// + relax).
enum { R_COMPUTE, R_UPPER, R_RELAX, R_XMEM, R_POLL, R_BMEM, R_XST };
__device__ constexpr int b7_role(int w)
{
    return w == 0 ? R_BMEM
         : w == 1 ? R_XMEM
         : w == 2 ? R_COMPUTE
         : w == 3 ? R_UPPER
         : w == 4 ? R_POLL
         : w == 5 ? R_RELAX
                  : R_XST;
}

namespace {

__device__ __forceinline__ double ld64(__amdgpu_buffer_rsrc_t rs,
                                       unsigned off)
{
    return buf_load<double>(rs, off);
}
__device__ __forceinline__ void st64(__amdgpu_buffer_rsrc_t rs, unsigned off,
                                     double v)
{
    buf_store<double, 0>(rs, off, v);
}
// keep a value in a vector register for the rest of the kernel
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

}  // namespace

struct B7Args {
    Grid g;
    int ntiles, njt, ns;   // tiles, j-tiles, boundary slices per tile
    const int2 *tiles;     // (j-tile, k-tile) per ticket
    const double *b;
    const double *xin;     // nullptr: start from zero
    double *xout;
    void *bnd;             // boundary store (records)
    int64_t bnd_elems;     // records
    unsigned epoch;
    uint64_t *ticket;
    uint64_t ticket_base;
    int *err;
    int spin_limit;
};

// C: device copy of the block constants (read once per launch).
template <bool BWD>
__global__ void __launch_bounds__(B7_NT)
    b7_tile_kernel(B7Args a, const Block7Consts *__restrict__ C)
{
    using R = Rec<double>;
    constexpr int KT = B7_KT;
    constexpr int NE = KT + 15;          // boundary rows per slice
    constexpr int WB = 5 * NE;           // records per slice
    constexpr int NH = 5 * (KT + 16);    // polled halo records
    constexpr int NXR = (KT + 2) * B7_RJ;
    constexpr int PS = B7_RJ * B7_RS;    // x-ring plane stride
    constexpr unsigned RB = R::bytes;
    extern __shared__ unsigned char smem_raw[];
    double *const xr = (double *)smem_raw;
    double *const br = xr + NXR * B7_RS;
    double *const ur = br + KT * B7_TJ * B7_BS;
    double *const gr = ur + KT * B7_TJ * B7_US;
    __shared__ int s_tile, s_abort;

    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int last = (int)a.g.size() - 1;
    const int tid = threadIdx.x, l = tid & 63;
    const int role = b7_role(tid >> 6);
    const int dir = BWD ? -1 : 1;
    const unsigned OOB = 0x80000000u;
    const int nbytes = (int)((unsigned)(last + 1) * 40u);
    const unsigned ep = a.epoch;

    // x-ring index of (plane kq, row jq), column 0, component 0
    auto xi = [](int kq, int jq) -> int {
        return ((kq + 1) * B7_RJ + (jq + 1)) * B7_RS;
    };
    // element index of sweep-order column 0, component 0 of row (j, k)
    auto rowbase = [&](int j, int k) -> int {
        const int v = (k * ny + j) * nx;
        return 5 * (BWD ? last - v : v);
    };

    if (tid == 0) s_abort = 0;
    int jt = 0, vt = 0, j0 = 0, k0 = 0, T0 = 0, T_start = 0, nblk = 0;
    // Every role runs this tile loop with the same barriers.
    auto next_tile = [&]() -> bool {
        __syncthreads();
        if (tid == 0) {
            uint64_t tk = atomicAdd((unsigned long long *)a.ticket, 1ull) -
                          a.ticket_base;
            s_tile = (tk < (uint64_t)a.ntiles && !s_abort) ? (int)tk : -1;
        }
        for (int e = tid; e < NXR * B7_RS; e += B7_NT) xr[e] = 0.0;
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0) return false;
        jt = a.tiles[tile].x;
        vt = a.tiles[tile].y;
        j0 = B7_TJ * jt;
        k0 = KT * vt;
        T0 = j0 + k0;
        T_start = T0 - 1 - B7_PRE;
        const int T_lastc = T0 + (B7_TJ - 1) + (KT - 1) + nx - 1;
        nblk = (T_lastc + 5 - T_start + 15) / 16;
        return true;
    };
    const __amdgpu_buffer_rsrc_t rs_b = __builtin_amdgcn_make_buffer_rsrc(
        a.bnd, 0, (int)(a.bnd_elems * RB), 0x00020000);

    if (role <= R_RELAX) {
        // ====== compute / upper / relax: lane = row (j0 + jj, k0 + kk) =====
        const int jj = l & 15, kk = l >> 4;
        double cf[3][25];
        double omb = 0.0;
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int e = 0; e < 25; ++e) {
                cf[v][e] = role == R_COMPUTE ? C->W[b7_lower_dir<BWD>(v)][e]
                           : role == R_UPPER ? C->B[b7_upper_dir<BWD>(v)][e]
                                             : (v == 0 ? C->G[e] : 0.0);
                pin(cf[v][e]);
            }
        if (role == R_RELAX) omb = C->omb;
        double *const own = xr + xi(kk, jj);
        double *const bown = br + (kk * B7_TJ + jj) * B7_BS;
        double *const uown = ur + (kk * B7_TJ + jj) * B7_US;
        double *const gown = gr + (kk * B7_TJ + jj) * B7_US;
        while (next_tile()) {
            const int j = j0 + jj, k = k0 + kk;
            const bool vc = j < ny && k < nz;
            const int sc = j + k;
            if (role == R_COMPUTE) {
                const int ipub =
                    jj == 15 ? kk : (kk == KT - 1 ? KT + jj : -1);
                const bool pub = vc && ipub >= 0;
                const int bout =
                    (vt * a.njt + jt) * a.ns * WB + ipub - T0 * WB;
                double xp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                for (int blk = 0; blk < nblk; ++blk) {
                    const int Tb = T_start + 16 * blk;
#pragma unroll 2
                    for (int ph = 0; ph < 16; ++ph) {
                        const int st = Tb + ph;
                        const int f = st - sc;
                        const int o = (f & (B7_W - 1)) * 5;
                        const int og = (f & 3) * 5;
                        double g[5], xn[3][5], x[5];
#pragma unroll
                        for (int c = 0; c < 5; ++c) {
                            g[c] = gown[og + c];
                            xn[0][c] = xp[c];                 // -x
                            xn[1][c] = own[o - B7_RS + c];    // -y
                            xn[2][c] = own[o - PS + c];       // -z
                        }
                        b7_lower(cf, g, xn, x);
                        const bool act = vc && (unsigned)f < (unsigned)nx;
                        if (act) {
#pragma unroll
                            for (int c = 0; c < 5; ++c) {
                                own[o + c] = x[c];
                                xp[c] = x[c];
                            }
                        }
                        const int rec = bout + st * WB;
#pragma unroll
                        for (int c = 0; c < 5; ++c)
                            R::store(rs_b,
                                     act && pub ? (unsigned)(rec + c * NE) * RB
                                                : OOB,
                                     R::make(x[c], ep));
                        __syncthreads();
                    }
                    if (s_abort) break;
                }
            } else if (role == R_UPPER) {
                for (int blk = 0; blk < nblk; ++blk) {
                    const int Tb = T_start + 16 * blk;
#pragma unroll 2
                    for (int ph = 0; ph < 16; ++ph) {
                        const int st = Tb + ph;
                        const int c = st - sc + 2;
                        const int ox = (c & (B7_W - 1)) * 5;
                        const int ox1 = ((c + 1) & (B7_W - 1)) * 5;
                        const int ob = (c & 7) * 5, ou = (c & 3) * 5;
                        double bv[5], xo[3][5], u[5];
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            bv[q] = bown[ob + q];
                            xo[0][q] = own[ox1 + q];          // +x
                            xo[1][q] = own[ox + B7_RS + q];   // +y
                            xo[2][q] = own[ox + PS + q];      // +z
                        }
                        b7_upper(cf, bv, xo, u);
#pragma unroll
                        for (int q = 0; q < 5; ++q) uown[ou + q] = u[q];
                        __syncthreads();
                    }
                    if (s_abort) break;
                }
            } else {
                for (int blk = 0; blk < nblk; ++blk) {
                    const int Tb = T_start + 16 * blk;
#pragma unroll 2
                    for (int ph = 0; ph < 16; ++ph) {
                        const int st = Tb + ph;
                        const int c = st - sc + 1;
                        const int ox = (c & (B7_W - 1)) * 5, ou = (c & 3) * 5;
                        double uv[5], xo[5], g[5];
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            uv[q] = uown[ou + q];
                            xo[q] = own[ox + q];
                        }
                        b7_relax(cf[0], omb, uv, xo, g);
#pragma unroll
                        for (int q = 0; q < 5; ++q) gown[ou + q] = g[q];
                        __syncthreads();
                    }
                    if (s_abort) break;
                }
            }
        }
    } else if (role == R_XMEM || role == R_BMEM || role == R_XST) {
        // ====== memory wavefronts ======
        // Per plane p (served at steps T with (T - T_start) mod 4 = p) and
        // element q the step-independent parts of the addresses: column
        // c = T + kc + lead, x- or b-ring index li + 5 (c mod ring), and
        // element index gb + 5 dir c (columns run backwards in memory in a
        // backward sweep, the 5 components of a point never do).  Rows
        // outside the grid get kc far below 0, so every column test fails
        // and their loads read 0; their ring slots hold 0.
        // The x staging, x store and b wavefronts run separate
        // instantiations of one loop (KIND 0, 1, 2): sharing one loop (and
        // its staging registers) behind a branch on the role made the
        // compiler wait, in every step, for the loads the other role would
        // have issued in the step before, which undid the 8-step prefetch.
        // The stores have a wavefront of their own because a wavefront keeps
        // at most 63 memory instructions in flight: with the stores, the x
        // staging loads could run only about 6 steps ahead.
        auto mem_role = [&](auto kind_tag) {
        constexpr int KIND = decltype(kind_tag)::value;
        constexpr bool xw = KIND != 2;
        const __amdgpu_buffer_rsrc_t rs_x = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.xin ? a.xin : a.b), 0, a.xin ? nbytes : 0, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs_bb = __builtin_amdgcn_make_buffer_rsrc(
            (void *)a.b, 0, nbytes, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs_o = __builtin_amdgcn_make_buffer_rsrc(
            (void *)a.xout, 0, nbytes, 0x00020000);
        constexpr int NOFF = -(1 << 28);
        double pipe[2][4][5], hpipe[2][4][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
#pragma unroll
                for (int q = 0; q < 5; ++q) pipe[h][p][q] = 0.0;
                hpipe[h][p][0] = hpipe[h][p][1] = 0.0;
            }
        const int plane_elems = 5 * ny * nx;  // elements per plane
        while (next_tile()) {
            // plane 0 of the tile; plane p adds p planes (uniform), and a
            // plane of rows at or past nz has no points
            int kc0[5], li0[5], gb0[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int e = l + 64 * q;
                const int jj = e / 20, o = e % 20;
                const int cq = o / 5, comp = o % 5;
                const int j = j0 + jj;
                kc0[q] = j < ny ? cq - (j + k0) : NOFF;
                li0[q] = xw ? xi(0, jj) + comp : jj * B7_BS + comp;
                gb0[q] = j < ny ? rowbase(j, k0) + comp : 0;
            }
            // halo elements (b wavefront): e < 20 row (16, p) of plane p;
            // 20 <= e < 100 plane 4, row 4p + (e - 20) / 20.  Between the
            // planes p the first kind moves one plane, the second 4 rows.
            int hkc0[2], hli0[2], hgb0[2], hm[2], hls[2], hgs[2], hj[2];
            bool hisa[2], hany[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = l + 64 * q;
                const bool isa = e < 20, ispl = e >= 20 && e < 100;
                const int r = isa ? 16 : (e - 20) / 20;
                const int o = isa ? e : (e - 20) % 20;
                const int hkk = isa ? 0 : KT;
                const int cq = o / 5, comp = o % 5;
                hisa[q] = isa;
                hany[q] = isa || ispl;
                hj[q] = j0 + r;
                hm[q] = isa ? 1 : 4;
                hls[q] = isa ? PS : 4 * B7_RS;
                hgs[q] = isa ? dir * plane_elems : dir * 20 * nx;
                hkc0[q] = cq - (j0 + r + k0 + hkk);
                hli0[q] = hany[q] ? xi(hkk, r) + comp : 0;
                hgb0[q] = rowbase(min(j0 + r, ny - 1), min(k0 + hkk, nz - 1)) +
                          comp;
                if (!isa && k0 + hkk >= nz) hgb0[q] = 0;
            }
            for (int blk = 0; blk < nblk; ++blk) {
                const int Tb = T_start + 16 * blk;
#pragma unroll 1
                for (int ph0 = 0; ph0 < 16; ph0 += 8)
#pragma unroll
                for (int s8 = 0; s8 < 8; ++s8) {
                    // plane p, pipeline half h: a load issued now is
                    // written to the ring 8 steps later
                    const int p = s8 & 3, h = s8 >> 2;
                    const int st = Tb + ph0 + s8;
                    const bool pin_k = k0 + p < nz;
                    if constexpr (xw) {
                        // store [f - 4, f) (KIND 1), stage [f + 4, f + 8)
                        // (KIND 0)
                        if constexpr (KIND == 1) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            const int kc = pin_k ? kc0[q] - p : NOFF;
                            const int li = li0[q] + p * PS;
                            const int gb = gb0[q] + p * dir * plane_elems;
                            const int cs = st + kc - 4;
                            const double xv = xr[li + (cs & (B7_W - 1)) * 5];
                            st64(rs_o,
                                 (unsigned)cs < (unsigned)nx
                                     ? (unsigned)(gb + dir * 5 * cs) * 8u
                                     : OOB,
                                 xv);
                        }
                        } else {
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            const int kc = pin_k ? kc0[q] - p : NOFF;
                            const int li = li0[q] + p * PS;
                            const int gb = gb0[q] + p * dir * plane_elems;
                            const int cx = st + kc + 4;
                            xr[li + (cx & (B7_W - 1)) * 5] = pipe[h][p][q];
                            const int cl = cx + 8;
                            pipe[h][p][q] = ld64(
                                rs_x, (unsigned)cl < (unsigned)nx
                                          ? (unsigned)(gb + dir * 5 * cl) * 8u
                                          : OOB);
                        }
                        }
                    } else {
                        // stage b [f + 3, f + 7)
#pragma unroll
                        for (int q = 0; q < 5; ++q) {
                            const int kc = pin_k ? kc0[q] - p : NOFF;
                            const int li = li0[q] + p * B7_TJ * B7_BS;
                            const int gb = gb0[q] + p * dir * plane_elems;
                            const int cb = st + kc + 3;
                            br[li + (cb & 7) * 5] = pipe[h][p][q];
                            const int cl = cb + 8;
                            pipe[h][p][q] = ld64(
                                rs_bb, (unsigned)cl < (unsigned)nx
                                           ? (unsigned)(gb + dir * 5 * cl) * 8u
                                           : OOB);
                        }
                        // old values of the halo rows, [f + 4, f + 8)
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const bool hv =
                                hany[q] &&
                                (hisa[q] ? hj[q] < ny && pin_k
                                         : hj[q] + 4 * p < ny && k0 + KT < nz);
                            const int kc = hv ? hkc0[q] - hm[q] * p : NOFF;
                            const int li = hli0[q] + p * hls[q];
                            const int gb = hgb0[q] + p * hgs[q];
                            const int ch = st + kc + 4;
                            if (hany[q])
                                xr[li + (ch & (B7_W - 1)) * 5] = hpipe[h][p][q];
                            const int cl = ch + 8;
                            hpipe[h][p][q] = ld64(
                                rs_x, (unsigned)cl < (unsigned)nx
                                          ? (unsigned)(gb + dir * 5 * cl) * 8u
                                          : OOB);
                        }
                    }
                    __syncthreads();
                }
                if (s_abort) break;
            }
        }
        };
        if (role == R_XMEM)
            mem_role(std::integral_constant<int, 0>{});
        else if (role == R_XST)
            mem_role(std::integral_constant<int, 1>{});
        else
            mem_role(std::integral_constant<int, 2>{});
    } else {
        // ====== poll wavefront: records l and l + 64 of the halo ======
        // halo row h < KT: (jj = -1, kk = h) from tile (jt - 1, vt), entry h;
        // h = KT + jj: plane k0 - 1 row jj from (jt, vt - 1), entry KT + jj
        // (jj < 15) or KT - 1 (jj = 15)
        typename R::V ppipe[B7_PRING][2];
#pragma unroll
        for (int p = 0; p < B7_PRING; ++p) ppipe[p][0] = ppipe[p][1] = R::V{};
        int spin_budget = a.spin_limit;
        while (next_tile()) {
            int hs[2], hslot[2], hT0[2], hx[2];
            bool hv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = l + 64 * q;
                // component-major, as the slices are laid out
                const int comp = e / (KT + 16), h = e % (KT + 16);
                const bool left = h < KT;
                const int jj = left ? -1 : h - KT;
                const int kk = left ? h : -1;
                const int j = j0 + jj, k = k0 + kk;
                const int pjt = left ? jt - 1 : jt, pvt = left ? vt : vt - 1;
                const int ent = left ? h : (jj < 15 ? KT + jj : KT - 1);
                hv[q] = e < NH && j >= 0 && j < ny && k >= 0 && k < nz;
                hs[q] = j + k;
                hT0[q] = B7_TJ * pjt + KT * pvt;
                hslot[q] = hv[q] ? (pvt * a.njt + pjt) * a.ns * WB +
                                       comp * NE + ent
                                 : 0;
                hx[q] = xi(hv[q] ? kk : 0, hv[q] ? jj : 0) + comp;
            }
            auto pslice = [&](int q, int T_) -> int {
                const int s = min(max(T_ - hT0[q], 0), a.ns - 1);
                return hslot[q] + s * WB;
            };
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
                                typename R::V r = ppipe[ph & (B7_PRING - 1)][q];
                                const unsigned src =
                                    (unsigned)pslice(q, st) * RB;
                                bool retried = false;
                                while (!R::ready(r, ep)) {
                                    retried = true;
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
                                    r = R::load(rs_b, src);
                                }
                                v = R::value(r);
                                // the consumer has caught up: the records
                                // preloaded before the wait are stale too
                                if (retried) {
#pragma unroll
                                    for (int d = 1; d < B7_POLL; ++d)
                                        ppipe[(ph + d) & (B7_PRING - 1)][q] =
                                            R::load(rs_b,
                                                    (unsigned)pslice(q, st + d) *
                                                        RB);
                                }
                            }
                            xr[hx[q] + (c & (B7_W - 1)) * 5] = v;
                        }
                        ppipe[(ph + B7_POLL) & (B7_PRING - 1)][q] = R::load(
                            rs_b, hv[q] ? (unsigned)pslice(q, st + B7_POLL) * RB
                                        : OOB);
                    }
                    __syncthreads();
                }
                if (s_abort) break;
            }
        }
    }
}

// ---------------------------------------------------------------- host --

B7Layout b7_layout(Grid g, int nw)
{
    B7Layout L{};
    L.nw = nw;
    L.kt = B7_KT;
    L.njt = (g.ny + B7_TJ - 1) / B7_TJ;
    L.nbands = (g.nz + L.kt - 1) / L.kt;
    L.ntiles = L.njt * L.nbands;
    L.ns = g.nx + (B7_TJ - 1) + (L.kt - 1);
    L.wb = 5 * (L.kt + 15);
    L.bnd_elems = (int64_t)L.ntiles * L.ns * L.wb;
    // tickets in the order of the tiles' first steps T0 = j0 + k0 (ties by
    // k): every dependence points to a smaller T0, and when there are more
    // tiles than workgroups, the tiles the front reaches first get the
    // workgroups first (lexicographic (k, j) order left tiles of small T0
    // to the second round: 162^3 half-sweep 0.608 -> 0.559 ms)
    for (int vt = 0; vt < L.nbands; ++vt)
        for (int jt = 0; jt < L.njt; ++jt) L.tiles.push_back(int2{jt, vt});
    std::stable_sort(L.tiles.begin(), L.tiles.end(),
                     [&](const int2 &x, const int2 &y) {
                         const int tx = B7_TJ * x.x + L.kt * x.y;
                         const int ty = B7_TJ * y.x + L.kt * y.y;
                         return tx != ty ? tx < ty : x.y < y.y;
                     });
    return L;
}

size_t b7_lds_bytes(int)
{
    return ((size_t)(B7_KT + 2) * B7_RJ * B7_RS +
            (size_t)B7_KT * B7_TJ * (B7_BS + 2 * B7_US)) *
           8;
}

int b7_threads(int) { return B7_NT; }

template <bool BWD>
static hipError_t b7_launch_t(const B7Args &a, const Block7Consts *C,
                              int grid, size_t lds, hipStream_t s)
{
    auto k = b7_tile_kernel<BWD>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
            160 * 1024 - 64);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(B7_NT), lds, s, a, C);
    return hipGetLastError();
}

hipError_t launch_sweep7(const m2s_stencil &A, const Block7Consts &C,
                         double omega, const void *b, const void *xin,
                         void *xout, bool bwd, Workspace &ws,
                         const SweepPlan &plan, hipStream_t s)
{
    (void)omega;  // built into C (set_block7_omega)
    // device copy of the block constants, refreshed when they change
    if (!ws.b7c) {
        hipError_t e = hipMalloc(&ws.b7c, sizeof(Block7Consts));
        if (e != hipSuccess) return e;
        ws.b7c_valid = false;
    }
    if (!ws.b7c_valid ||
        std::memcmp(&ws.b7c_host, &C, sizeof(Block7Consts)) != 0) {
        // ordered on the sweep's stream: after the sweeps already queued
        // there (which may still read the old constants), before this one;
        // the wait for the copy keeps the host source valid until it is
        // read (the constants change only with the blocks or omega)
        std::memcpy(&ws.b7c_host, &C, sizeof(Block7Consts));
        hipError_t e = hipMemcpyAsync(ws.b7c, &ws.b7c_host,
                                      sizeof(Block7Consts),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            ws.b7c_valid = false;
            return e;
        }
        ws.b7c_valid = true;
    }
    const size_t lds = b7_lds_bytes(1);
    const uint64_t base = ws.ticket_base;
    ws.ticket_base += (uint64_t)plan.nslabs + (uint64_t)plan.grid;
    if (++ws.epoch == 0) ++ws.epoch;
    B7Args a{};
    a.g = Grid{A.ext.nx, A.ext.ny, A.ext.nz};
    a.ntiles = plan.nslabs;
    a.njt = ws.tile_nutb;
    a.ns = ws.tile_ns;
    a.tiles = ws.tile_list;
    a.b = (const double *)b;
    a.xin = (const double *)xin;
    a.xout = (double *)xout;
    a.bnd = ws.bnd;
    a.bnd_elems = ws.bnd_elems;
    a.epoch = ws.epoch;
    a.ticket = ws.ticket;
    a.ticket_base = base;
    a.err = ws.err;
    const char *e = getenv("M2S_SPIN_LIMIT");
    a.spin_limit = e ? std::max(1, atoi(e)) : (1 << 22);
    const Block7Consts *cd = (const Block7Consts *)ws.b7c;
    return bwd ? b7_launch_t<true>(a, cd, plan.grid, lds, s)
               : b7_launch_t<false>(a, cd, plan.grid, lds, s);
}

}  // namespace m2s
