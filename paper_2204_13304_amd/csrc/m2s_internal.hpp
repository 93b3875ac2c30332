// m2s_internal.hpp -- types and device helpers shared by the HIP kernels and
// the host side of libm2s.so.  Not part of the public ABI (include/m2s.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "../../include/m2s.h"

namespace m2s {

// Grid with x fastest: p = (k*ny + j)*nx + i.
struct Grid {
    int nx, ny, nz;
    __host__ __device__ int64_t idx(int i, int j, int k) const
    {
        return ((int64_t)k * ny + j) * nx + i;
    }
    __host__ __device__ int64_t size() const { return (int64_t)nx * ny * nz; }
    __host__ __device__ bool in(int i, int j, int k) const
    {
        return i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
    }
};

// A backward sweep is a forward sweep in reflected ("virtual") coordinates
// iv = nx-1-i, jv = ny-1-j, kv = nz-1-k.  Every kernel works in virtual
// coordinates and maps to memory through this helper.
template <bool BWD>
struct Virt {
    Grid g;
    __device__ int64_t idx(int iv, int jv, int kv) const
    {
        return BWD ? g.idx(g.nx - 1 - iv, g.ny - 1 - jv, g.nz - 1 - kv)
                   : g.idx(iv, jv, kv);
    }
    __device__ int ri(int iv) const { return BWD ? g.nx - 1 - iv : iv; }
    __device__ int rj(int jv) const { return BWD ? g.ny - 1 - jv : jv; }
    __device__ int rk(int kv) const { return BWD ? g.nz - 1 - kv : kv; }
};

// Face-array addressing of the VAR7 operator.
struct Faces {
    int nx, ny, nz;
    __host__ __device__ int64_t ix(int i, int j, int k) const
    {
        return ((int64_t)k * ny + j) * (nx + 1) + i;
    }
    __host__ __device__ int64_t iy(int i, int j, int k) const
    {
        return ((int64_t)k * (ny + 1) + j) * nx + i;
    }
    __host__ __device__ int64_t iz(int i, int j, int k) const
    {
        return ((int64_t)k * ny + j) * nx + i;
    }
    __host__ __device__ int64_t nfx() const { return (int64_t)nz * ny * (nx + 1); }
    __host__ __device__ int64_t nfy() const { return (int64_t)nz * (ny + 1) * nx; }
    __host__ __device__ int64_t nfz() const { return (int64_t)(nz + 1) * ny * nx; }
};

// BLOCK7 constants: the seven 5x5 blocks B_d (order C, -x, +x, -y, +y, -z,
// +z; row-major), the LU factorisation with partial pivoting of the centre
// block D = B_0 (unit lower L below the diagonal, U on and above; inverse
// pivots precomputed), and for the relaxation factor w of a block SSOR
// sweep W_d = w D^{-1} B_d (d = 1..6), G = w D^{-1} and 1 - w.
struct Block7Consts {
    double B[7][25];
    double lu[25];
    double inv_udiag[5];
    int piv[5];
    double W[7][25];
    double G[25];
    double omb;    // 1 - w
    double omega;  // w
};

// Wavefront schedule of one sweep (see the sweep kernel for its meaning).
struct SweepPlan {
    int slab_planes;  // planes per tile (4 per compute wavefront)
    int nslabs;       // tiles
    int row_slots;    // rows per tile and plane
    int lag_row;      // step weight of a row (2 for 27 points: T = i+2u+2k)
    int lag_plane;    // step weight of a plane
    int threads;      // workgroup size
    int publish_every;  // boundary records are written every step: 1
    int grid;         // workgroups launched (<= tiles)
};

// x_i = (r_i - off * (S + x_new(i-1))) / diag, evaluated as
//   B  = (F(i-1) + F(i)) + (A(i+1) + x_old(i+1))
//   S  = B + D(i+1)
//   x_i = fma(-off, S, fma(-off, x_new(i-1), r_i)) * (1 / diag),
// the association of every 27-point sweep kernel (the sequential one and
// the tiled wavefront one use this same function).
template <typename T>
__device__ __forceinline__ T c27_combine(T r, T B, T Dp, T xn_prev, T off,
                                         T inv_diag)
{
    const T S = B + Dp;
    const T t1 = fma(-off, xn_prev, r);
    return fma(-off, S, t1) * inv_diag;
}

// VAR7 point update x_p = (r_p + sum_d k_d x_q) / (sum_d k_d) over the six
// faces in real orientation (m: the face towards -x, p: towards +x, ...);
// neighbours outside the grid enter as 0.  The sequential and the tiled
// sweep kernels both call this function, so their results agree bitwise.
template <typename T>
__device__ __forceinline__ T v7_combine(T r, T vmx, T vpx, T vmy, T vpy,
                                        T vmz, T vpz, T kxm, T kxp, T kym,
                                        T kyp, T kzm, T kzp)
{
    const T s1 = fma(kxm, vmx, kxp * vpx);
    const T s2 = fma(kym, vmy, kyp * vpy);
    const T s3 = fma(kzm, vmz, kzp * vpz);
    const T S = (s1 + s2) + s3;
    const T d = ((kxm + kxp) + (kym + kyp)) + (kzm + kzp);
    return (r + S) / d;
}

// One block-SSOR point (the NPB-LU-shaped BLOCK7x5 operator, Sec. 7.1),
//   x = (1 - w) x_old + w D^{-1} (b - sum over neighbours q of B_d x_q),
// in three parts.  Directions are taken in sweep order: the sweep's lower
// neighbours (-x, -y, -z) already hold new values, the upper ones (+x, +y,
// +z) old values; in a backward sweep the sweep's -x is the grid's +x, so
// it takes the +x block.
//   u = b - sum_{upper d} B_d x_d                     (b7_upper)
//   g = (1 - w) x_old + G u,        G = w D^{-1}       (b7_relax)
//   x = g - sum_{lower d} W_d x_d,  W_d = w D^{-1} B_d  (b7_lower)
// Only the last part needs the values of the previous wavefront step.
// Neighbours outside the grid enter as 0.  The sequential and the tiled
// sweep kernels both call these functions, so their results agree bitwise.
// v = 0, 1, 2 is the sweep's x, y, z direction.
template <bool BWD>
__host__ __device__ constexpr int b7_lower_dir(int v)
{
    return BWD ? 2 * v + 2 : 2 * v + 1;
}
template <bool BWD>
__host__ __device__ constexpr int b7_upper_dir(int v)
{
    return BWD ? 2 * v + 1 : 2 * v + 2;
}

// Bu[v]: the block of upper direction v; xo[v]: that neighbour's values.
// One partial sum per direction (short independent chains), subtracted in
// the order x, y, z.
__device__ __forceinline__ void b7_upper(const double (&Bu)[3][25],
                                         const double (&b)[5],
                                         const double (&xo)[3][5],
                                         double (&u)[5])
{
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double t[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            t[v] = Bu[v][5 * a] * xo[v][0];
#pragma unroll
            for (int c = 1; c < 5; ++c)
                t[v] = fma(Bu[v][5 * a + c], xo[v][c], t[v]);
        }
        u[a] = ((b[a] - t[0]) - t[1]) - t[2];
    }
}

__device__ __forceinline__ void b7_relax(const double (&G)[25], double omb,
                                         const double (&u)[5],
                                         const double (&xold)[5],
                                         double (&g)[5])
{
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double t = G[5 * a] * u[0];
#pragma unroll
        for (int c = 1; c < 5; ++c) t = fma(G[5 * a + c], u[c], t);
        g[a] = fma(omb, xold[a], t);
    }
}

// Wl[v]: W of lower direction v; xn[v]: that neighbour's new values.  The
// -x part starts from g (its value is the lane's own result of the previous
// step); the -y and -z parts, whose values arrive last, are separate short
// chains subtracted at the end.
__device__ __forceinline__ void b7_lower(const double (&Wl)[3][25],
                                         const double (&g)[5],
                                         const double (&xn)[3][5],
                                         double (&x)[5])
{
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double s0 = g[a];
#pragma unroll
        for (int c = 0; c < 5; ++c) s0 = fma(-Wl[0][5 * a + c], xn[0][c], s0);
        double t[2];
#pragma unroll
        for (int v = 1; v < 3; ++v) {
            t[v - 1] = Wl[v][5 * a] * xn[v][0];
#pragma unroll
            for (int c = 1; c < 5; ++c)
                t[v - 1] = fma(Wl[v][5 * a + c], xn[v][c], t[v - 1]);
        }
        x[a] = (s0 - t[0]) - t[1];
    }
}

// Workspace (opaque in the ABI).
struct Workspace {
    m2s_kind kind;
    m2s_dtype dtype;
    Grid g;
    int dev;
    uint64_t *ticket;   // ticket counter (monotone)
    int *err;           // device error latch
    void *scratch;      // one vector of the stencil's size
    void *scratch2;     // second vector (adjoint chains)
    void *bnd;          // tiled sweeps: tile boundary store (records)
    int64_t bnd_elems;  // records
    int tile_nw;        // compute wavefronts per tile of the layout
    int tile_ntiles;
    int tile_nutb;      // boundary-store tile slots per k-tile
    int tile_ns;        // boundary slices per tile
    int2 *tile_list;    // 27-point: (u-tile, k-tile) per ticket, device
    void *b7c;          // block SSOR: device copy of the block constants
    Block7Consts b7c_host;
    bool b7c_valid;
    uint32_t epoch;
    uint64_t ticket_base;
};

constexpr int kErrTimeout = 1;

}  // namespace m2s

// Internal launchers implemented in the .hip files (C++ linkage, not ABI).
namespace m2s {
hipError_t launch_spmv(const m2s_stencil &A, const void *x, void *y,
                       hipStream_t s);
hipError_t launch_spmv_part(const m2s_stencil &A, int part, const void *x,
                            void *y, hipStream_t s);
hipError_t launch_sweep(const m2s_stencil &A, const Block7Consts *b7,
                        double omega, const void *r, const void *xin,
                        void *xout, bool bwd, bool zero_init, Workspace &ws,
                        const SweepPlan &plan, hipStream_t s);
hipError_t launch_sweep_sequential(const m2s_stencil &A, const void *r,
                                   void *x, bool bwd, hipStream_t s);
hipError_t launch_restrict(const m2s_stencil &A, const void *r,
                           const void *z, void *rc, hipStream_t s);
hipError_t launch_prolong(const m2s_stencil &Afine, const void *zc, void *z,
                          hipStream_t s);
hipError_t launch_var7_coarsen(m2s_dtype t, Grid fine, const void *kx,
                               const void *ky, const void *kz, void *kxc,
                               void *kyc, void *kzc, hipStream_t s);
hipError_t launch_face_grad(Grid g, const double *u, const double *lam,
                            double *gx, double *gy, double *gz,
                            hipStream_t s);
hipError_t launch_convert(const void *src, m2s_dtype st, void *dst,
                          m2s_dtype dt, int64_t n, hipStream_t s);
hipError_t launch_fill(void *dst, m2s_dtype t, int64_t n, double v,
                       hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t bytes,
                       hipStream_t s);
hipError_t launch_scale(void *x, m2s_dtype t, int64_t n, double a,
                        hipStream_t s);
// x += y
hipError_t launch_add(void *x, const void *y, m2s_dtype t, int64_t n,
                      hipStream_t s);

// 27-point wavefront sweep (k_sweep27.hip).
hipError_t launch_sweep27(const m2s_stencil &A, const void *r,
                          const void *xin, void *xout, bool bwd,
                          Workspace &ws, const SweepPlan &plan,
                          hipStream_t s);
// The FP32 backward sweep (from xin) storing its result widened to FP64.
hipError_t launch_sweep27_wide(const m2s_stencil &A, const void *r,
                               const void *xin, double *xout, Workspace &ws,
                               const SweepPlan &plan, hipStream_t s);
// Tiling of the 27-point sweep: tiles of 16 u = j + k by 4 * nw planes.
struct C27Layout {
    int nw, kt, nbands, nutb, ns, wb;
    int64_t bnd_elems;
    std::vector<int2> tiles;  // valid tiles in ticket order
};
C27Layout c27_layout(Grid g, int nw);
size_t c27_lds_bytes(int nw, m2s_dtype t, int mode);
// ILU of the 27-point operator on the same tiles (F64): mode 1 factor
// (out = w = 1/d), 2 lower solve (out = y from r), 3 upper solve (out = z
// from r = y); w is the factor's weight array for modes 2 and 3.
hipError_t launch_dilu27(const m2s_stencil &A, int mode, const void *r,
                        const void *w, void *out, Workspace &ws,
                        const SweepPlan &plan, hipStream_t s);
int c27_threads(int nw);  // nw compute + nw memory + 1 poll wavefronts
// ILU(0) of the 27-point operator, hyperplane by hyperplane (k_ilu0.hip):
// L (13 per point), U (14 per point), z = (L U)^{-1} r.
hipError_t launch_ilu0_factor(const m2s_stencil &A, double *L, double *U,
                              hipStream_t s);
hipError_t launch_ilu0_apply(const m2s_stencil &A, const double *L,
                             const double *U, const double *r, double *z,
                             hipStream_t s);
// The band-wavefront solves: bands of kt planes (ny * kt <= 512 rows, one
// lane each), coefficients packed by the band's steps (k_ilu0.hip).
struct IlbLayout {
    int kt = 0, nbands = 0, nsteps = 0, threads = 0;  // kt = 0: ny > 512
    size_t lds = 0;
    std::vector<int> doff;   // first packed index of each plane diagonal
};
IlbLayout ilb_layout(const Grid &g);
hipError_t launch_ilu0_pack(const m2s_stencil &A, const int *doff,
                            const double *L, const double *U, double *Lp,
                            double *Up, hipStream_t s);
hipError_t launch_ilu0_apply_packed(const m2s_stencil &A, const IlbLayout &L,
                                    const int *doff, const double *Lp,
                                    const double *Up, const double *r,
                                    double *y, double *t, double *z,
                                    Workspace &ws, void *rec,
                                    int64_t rec_elems, hipStream_t s);
// Tiling of the block SSOR sweep: rectangular tiles of 16 j by 4 * nw k.
struct B7Layout {
    int nw, kt, njt, nbands, ntiles, ns, wb;
    int64_t bnd_elems;
    std::vector<int2> tiles;  // (j-tile, k-tile) per ticket
};
B7Layout b7_layout(Grid g, int nw);
size_t b7_lds_bytes(int nw);
int b7_threads(int nw);  // seven wavefronts, one per role
hipError_t launch_sweep7(const m2s_stencil &A, const Block7Consts &C,
                         double omega, const void *b, const void *xin,
                         void *xout, bool bwd, Workspace &ws,
                         const SweepPlan &plan, hipStream_t s);

// Tiling of the VAR7 sweep (k_sweep7v.hip): the same rectangular tiles,
// one boundary record per row.
using V7Layout = B7Layout;
V7Layout v7_layout(Grid g, int nw);
size_t v7_lds_bytes(int nw, m2s_dtype t);
int v7_threads(int nw);  // nw compute + nw memory + 1 poll wavefronts
hipError_t launch_sweep7v(const m2s_stencil &A, const void *r,
                          const void *xin, void *xout, bool bwd,
                          Workspace &ws, const SweepPlan &plan,
                          hipStream_t s);

// Jacobi iterations of the 2-D 9-point operator, temporally blocked
// (k_jacobi.hip); the result ends in x, tmp is a second nx*ny buffer.
hipError_t launch_jacobi9(int nx, int ny, double diag, double off,
                          const double *b, double *x, double *tmp, int iters,
                          int tblock, hipStream_t s);

// Pentadiagonal line solves along one axis (k_lines.hip); work: 2n doubles.
hipError_t launch_penta_lines(int nx, int ny, int nz, int axis,
                              const double *coef, const double *r, double *x,
                              double *work, hipStream_t s);
hipError_t launch_bt_lines(int nx, int ny, int nz, int axis,
                           const double *coef, const double *r, double *x,
                           double *work, hipStream_t s);

// bytes of one boundary record: the value and the launch epoch
inline size_t c27_record_bytes(m2s_dtype t) { return t == M2S_F64 ? 16 : 8; }

// CG vector kernels (double).  Scalars live in a small device array `sc`.
// SC_BD latches a breakdown (p.Ap <= 0 or a non-finite r.z, p.Ap) on the
// device, so that a solve need not read the scalars back every iteration;
// SC_BDIT holds the iteration that latched it.  From that iteration on the
// update kernels leave x, r and p as they are.
enum CgScalar {
    SC_RZ = 0, SC_RZ_OLD, SC_PAP, SC_RR, SC_BD, SC_BDIT, SC_N
};
int dot_partials_capacity();
hipError_t launch_dot(const double *x, const double *y, int64_t n,
                      double *partials, double *out, hipStream_t s);
hipError_t launch_dot_reset(double *partials, hipStream_t s);
hipError_t launch_stream(int kind, const double *a, const double *b,
                         double *c, double sc, int64_t n, hipStream_t s);
// r = b - Ax (Ax given) and rr = r.r
hipError_t launch_residual(const double *b, const double *ax, double *r,
                           int64_t n, double *partials, double *rr_out,
                           hipStream_t s);
// p = z (first) or p = z + (rz/rz_old) p ; rz computed beforehand
hipError_t launch_update_p(const double *z, double *p, int64_t n,
                           const double *sc, bool first, hipStream_t s);
// x += alpha p ; r -= alpha Ap ; rr = r.r ; alpha = rz / pAp
hipError_t launch_update_xr(double *x, double *r, const double *p,
                            const double *ap, int64_t n, double *sc,
                            double *partials, int iter, hipStream_t s);
// Ap = A p and pAp = p.Ap fused (CONST27/VAR7 double)
hipError_t launch_spmv_dot(const m2s_stencil &A, const double *p, double *ap,
                           double *partials, double *out, hipStream_t s);
// x = 0 with a small fill kernel (graph-capture safe)
}  // namespace m2s
