// k_sweep.hip -- per-point arithmetic of the exact lexicographic Gauss-
// Seidel / block-SSOR half-sweeps (the Seidel-style stencils of the paper,
// Sec. 2.1.2 and Sec. 4.3.3), the one-thread sequential kernel built from
// it (the reference order every wavefront kernel must reproduce bitwise),
// and the routing of a half-sweep to the tiled wavefront kernel of its
// stencil kind (k_sweep27.hip, k_sweep7v.hip, k_sweep7.hip).
//
// Half-sweeps are out of place: new values go to x_out, so a point reads
// its lower (already updated) neighbours from x_out and its upper
// neighbours from x_in; there is no write-after-read hazard and the result
// equals the in-place lexicographic sweep exactly.
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
    return v7_combine<T>(r[g.idx(i, j, k)], vmx, vpx, vmy, vpy, vmz, vpz,
                         kxm, kxp, kym, kyp, kzm, kzp);
}

// BLOCK7: x_p <- (1-w) x_p + w D^{-1} (b_p - sum_{d=1..6} B_d x_{p+d}),
// through b7_upper / b7_relax / b7_lower (the relaxation factor is built
// into the constants).
template <bool BWD>
__device__ __forceinline__ void b7_point(const Virt<BWD> &V,
                                         const Block7Consts &C,
                                         const double *b, const double *xn,
                                         const double *xo, double *out,
                                         int iv, int jv, int kv)
{
    // sweep coordinates: (iv, jv, kv) - 1 are updated, + 1 are not
    const Grid &g = V.g;
    const int64_t p = V.idx(iv, jv, kv);
    const int di[3] = {1, 0, 0};
    const int dj[3] = {0, 1, 0};
    const int dk[3] = {0, 0, 1};
    double xu[3][5], xl[3][5], bb[5], old[5], u[5], gg[5], res[5];
    double Bu[3][25], Wl[3][25];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int iu = iv + di[v], ju = jv + dj[v], ku = kv + dk[v];
        const int il = iv - di[v], jl = jv - dj[v], kl = kv - dk[v];
        const bool hu = g.in(iu, ju, ku), hl = g.in(il, jl, kl);
        const int64_t qu = hu ? 5 * V.idx(iu, ju, ku) : 0;
        const int64_t ql = hl ? 5 * V.idx(il, jl, kl) : 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            xu[v][c] = (hu && xo) ? xo[qu + c] : 0.0;
            xl[v][c] = hl ? xn[ql + c] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 25; ++e) {
            Bu[v][e] = C.B[b7_upper_dir<BWD>(v)][e];
            Wl[v][e] = C.W[b7_lower_dir<BWD>(v)][e];
        }
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        bb[a] = b[5 * p + a];
        old[a] = xo ? xo[5 * p + a] : 0.0;
    }
    b7_upper(Bu, bb, xu, u);
    b7_relax(C.G, C.omb, u, old, gg);
    b7_lower(Wl, gg, xl, res);
#pragma unroll
    for (int a = 0; a < 5; ++a) out[5 * p + a] = res[a];
}

// --------------------------------------------------------------------------
// Kernel arguments.
// --------------------------------------------------------------------------
template <typename T>
struct SweepArgs {
    Grid g;
    const T *r;
    const T *xin;   // nullptr: start from zero
    T *xout;
    // CONST27
    T off, inv_diag;
    // VAR7
    const T *kx, *ky, *kz;
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
        b7_point<BWD>(V, b7, (const double *)a.r, (const double *)a.xout,
                      (const double *)a.xin, (double *)a.xout, iv, jv, kv);
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
        return launch_sweep7v(A, r, xin, xout, bwd, ws, plan, s);
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

}  // namespace m2s
