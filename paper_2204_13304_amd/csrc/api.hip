// api.hip -- host side of libm2s.so: the extern "C" entry points declared in
// include/m2s.h.  Validates arguments, plans the wavefront sweep, owns the
// workspace and multigrid objects, and drives the PCG loop.  Every
// arithmetic step runs in the HIP kernels of k_sweep.hip / k_ops.hip.
#include "m2s_internal.hpp"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

using namespace m2s;

namespace m2s {
hipError_t launch_sweep_sequential_b7(const m2s_stencil &A,
                                      const Block7Consts &b7, double omega,
                                      const void *b, void *x, bool bwd,
                                      hipStream_t s);
// k_xline.hip: line-scheduled 27-point half-sweep with the x-line scan
// (FP64); rec holds one 16-byte record per point.
size_t xline_lds_bytes(int nx);
hipError_t launch_xline_sweep(const m2s_stencil &A, const void *r,
                              const void *xin, void *xout, bool bwd,
                              Workspace &ws, void *rec, hipStream_t s);

// LU with partial pivoting of the 5x5 centre block (row-major), host side.
hipError_t fill_block7_consts(const double *blocks, Block7Consts &C)
{
    if (!blocks) return hipErrorInvalidValue;
    for (int d = 0; d < 7; ++d)
        for (int e = 0; e < 25; ++e) C.B[d][e] = blocks[25 * d + e];
    double a[25];
    for (int e = 0; e < 25; ++e) a[e] = blocks[e];
    for (int c = 0; c < 5; ++c) {
        int p = c;
        double best = std::fabs(a[5 * c + c]);
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(a[5 * r + c]) > best) {
                best = std::fabs(a[5 * r + c]);
                p = r;
            }
        if (!(best > 0.0) || !std::isfinite(best)) return hipErrorInvalidValue;
        C.piv[c] = p;
        if (p != c)
            for (int t = 0; t < 5; ++t) std::swap(a[5 * c + t], a[5 * p + t]);
        for (int r = c + 1; r < 5; ++r) {
            a[5 * r + c] /= a[5 * c + c];
            for (int t = c + 1; t < 5; ++t)
                a[5 * r + t] -= a[5 * r + c] * a[5 * c + t];
        }
    }
    for (int e = 0; e < 25; ++e) C.lu[e] = a[e];
    for (int c = 0; c < 5; ++c) C.inv_udiag[c] = 1.0 / a[5 * c + c];
    return hipSuccess;
}

// The relaxation-factor products of a block SSOR sweep: D^{-1} column by
// column from the LU factors (rows swapped as in the factorisation, then
// forward and back substitution), G = w D^{-1}, W_d = w D^{-1} B_d.
void set_block7_omega(Block7Consts &C, double omega)
{
    double Dinv[25];
    for (int col = 0; col < 5; ++col) {
        double y[5] = {0, 0, 0, 0, 0};
        y[col] = 1.0;
        for (int c = 0; c < 5; ++c)
            if (C.piv[c] != c) std::swap(y[c], y[C.piv[c]]);
        for (int r = 1; r < 5; ++r)
            for (int c = 0; c < r; ++c) y[r] -= C.lu[5 * r + c] * y[c];
        for (int r = 4; r >= 0; --r) {
            for (int c = r + 1; c < 5; ++c) y[r] -= C.lu[5 * r + c] * y[c];
            y[r] *= C.inv_udiag[r];
        }
        for (int r = 0; r < 5; ++r) Dinv[5 * r + col] = y[r];
    }
    for (int e = 0; e < 25; ++e) C.G[e] = omega * Dinv[e];
    for (int e = 0; e < 25; ++e) C.W[0][e] = 0.0;
    for (int d = 1; d < 7; ++d)
        for (int r = 0; r < 5; ++r)
            for (int c = 0; c < 5; ++c) {
                double t = 0.0;
                for (int q = 0; q < 5; ++q)
                    t += Dinv[5 * r + q] * C.B[d][5 * q + c];
                C.W[d][5 * r + c] = omega * t;
            }
    C.omb = 1.0 - omega;
    C.omega = omega;
}
}  // namespace m2s

struct m2s_workspace : public Workspace {
    // line-scheduled 27-point sweep: one 16-byte record per point, made on
    // the first such call (zeroed: epoch 0 is never a launch's)
    void *xl_rec = nullptr;
    // band-wavefront ILU(0) solves: the packed layout's diagonal offsets
    int *ilb_doff = nullptr;
    int ilb_nd = 0;
};

namespace {


int env_int(const char *name, int dflt)
{
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

size_t elem_size(const m2s_stencil &A)
{
    size_t e = A.dtype == M2S_F64 ? 8 : 4;
    return A.kind == M2S_BLOCK7_5 ? 5 * e : e;
}

int64_t npoints(const m2s_stencil &A)
{
    return (int64_t)A.ext.nx * A.ext.ny * A.ext.nz;
}

m2s_status validate(const m2s_stencil *A)
{
    if (!A) return M2S_ERR_ARG;
    if (A->kind != M2S_CONST27 && A->kind != M2S_VAR7 &&
        A->kind != M2S_BLOCK7_5)
        return M2S_ERR_ARG;
    if (A->dtype != M2S_F64 && A->dtype != M2S_F32) return M2S_ERR_DTYPE;
    if (A->ext.nx <= 0 || A->ext.ny <= 0 || A->ext.nz <= 0)
        return M2S_ERR_SHAPE;
    if (npoints(*A) > ((int64_t)1 << 40)) return M2S_ERR_SHAPE;
    if (A->kind == M2S_VAR7 && (!A->kx || !A->ky || !A->kz))
        return M2S_ERR_ARG;
    if (A->kind == M2S_BLOCK7_5) {
        if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
        if (!A->blocks) return M2S_ERR_ARG;
    }
    if (A->kind == M2S_CONST27 && !(A->diag != 0.0 && std::isfinite(A->diag)))
        return M2S_ERR_ARG;
    return M2S_OK;
}

bool overlap(const void *a, const void *b, size_t bytes)
{
    if (!a || !b) return false;
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

// [a, a + na) and [b, b + nb) share a byte
bool overlap2(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b) return false;
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

m2s_status hip_status(hipError_t e)
{
    return e == hipSuccess ? M2S_OK : M2S_ERR_HIP;
}

#define M2S_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return M2S_ERR_HIP;       \
    } while (0)

// The wavefront schedule: tiles of 16 rows by 4 * nw planes, one lane per
// row; point (i, j, k) runs at step i + lag_row*j + lag_plane*k within its
// tile (the hyperplane of Sec. 6.1.3; rows u = j + k for 27 points).
m2s_status make_plan(const m2s_stencil &A, SweepPlan &P, bool with_grid)
{
    const int nx = A.ext.nx, ny = A.ext.ny, nz = A.ext.nz;
    const bool c27 = A.kind == M2S_CONST27;
    P.lag_row = c27 ? 2 : 1;
    P.lag_plane = c27 ? 4 : 1;
    if (c27) {
        // tiles of 16 u = j + k rows by 4 * nw planes, one lane per row;
        // buffer loads address a vector with 32-bit byte offsets
        if ((int64_t)nx * ny * nz * elem_size(A) >= ((int64_t)1 << 31))
            return M2S_ERR_SHAPE;
        // 2 compute wavefronts (8 planes) per tile: with the memory and poll
        // wavefronts that is 5 per CU; 4 compute wavefronts halve the tile
        // crossings along k but put 3 wavefronts on a SIMD
        int nw = env_int("M2S_C27_WAVES", 2);
        if (nw != 1 && nw != 2 && nw != 4) nw = 2;
        const C27Layout L = c27_layout(Grid{nx, ny, nz}, nw);
        if (L.bnd_elems * (int64_t)c27_record_bytes(A.dtype) >=
            ((int64_t)1 << 31))
            return M2S_ERR_SHAPE;
        P.row_slots = 16;
        P.slab_planes = L.kt;
        P.nslabs = (int)L.tiles.size();
        P.threads = c27_threads(nw);
        P.publish_every = 1;
        P.grid = 0;
        if (with_grid) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess) return M2S_ERR_HIP;
            if (hipDeviceGetAttribute(&cus,
                                      hipDeviceAttributeMultiprocessorCount,
                                      dev) != hipSuccess)
                return M2S_ERR_HIP;
            // one tile per CU: a CU holds one tile's rings anyway for
            // nw = 4, and spinning tiles should not share a CU with
            // working ones
            const int per_cu = std::max(1, env_int("M2S_C27_PER_CU", 1));
            P.grid = std::max(1, std::min(P.nslabs, cus * per_cu));
        }
        return M2S_OK;
    } else if (A.kind == M2S_VAR7) {
        // rectangular tiles of 16 j by 4 * nw k, one lane per row; buffer
        // loads address x, r and the face arrays with 32-bit byte offsets
        const int64_t es = elem_size(A);
        if ((int64_t)nz * ny * (nx + 1) * es >= ((int64_t)1 << 31) ||
            (int64_t)nz * (ny + 1) * nx * es >= ((int64_t)1 << 31) ||
            (int64_t)(nz + 1) * ny * nx * es >= ((int64_t)1 << 31))
            return M2S_ERR_SHAPE;
        // one compute wavefront (4 planes) per tile measured fastest: the
        // tile's step is short, so more tiles in flight beat fewer crossings
        int nw = env_int("M2S_V7_WAVES", 1);
        if (nw != 1 && nw != 2 && nw != 4) nw = 1;
        const V7Layout L = v7_layout(Grid{nx, ny, nz}, nw);
        if (L.bnd_elems * (int64_t)c27_record_bytes(A.dtype) >=
            ((int64_t)1 << 31))
            return M2S_ERR_SHAPE;
        P.row_slots = 16;
        P.slab_planes = L.kt;
        P.nslabs = L.ntiles;
        P.threads = v7_threads(nw);
        P.publish_every = 1;
        P.grid = 0;
        if (with_grid) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess) return M2S_ERR_HIP;
            if (hipDeviceGetAttribute(&cus,
                                      hipDeviceAttributeMultiprocessorCount,
                                      dev) != hipSuccess)
                return M2S_ERR_HIP;
            P.grid = std::max(1, std::min(P.nslabs, cus));
        }
        return M2S_OK;
    } else if (A.kind == M2S_BLOCK7_5) {
        // rectangular tiles of 16 j by 4 * nw k, one lane per row
        if ((int64_t)nx * ny * nz * 40 >= ((int64_t)1 << 31))
            return M2S_ERR_SHAPE;
        // tiles of 16 j by 4 k: six wavefronts (compute, the two helpers
        // that run ahead of it, two memory wavefronts, poll), each of the
        // arithmetic ones holding its 75 block coefficients in registers
        const int nw = 1;
        const B7Layout L = b7_layout(Grid{nx, ny, nz}, nw);
        if (L.bnd_elems * 16 >= ((int64_t)1 << 31)) return M2S_ERR_SHAPE;
        P.row_slots = 16;
        P.slab_planes = L.kt;
        P.nslabs = L.ntiles;
        P.threads = b7_threads(nw);
        P.publish_every = 1;
        P.grid = 0;
        if (with_grid) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess) return M2S_ERR_HIP;
            if (hipDeviceGetAttribute(&cus,
                                      hipDeviceAttributeMultiprocessorCount,
                                      dev) != hipSuccess)
                return M2S_ERR_HIP;
            P.grid = std::max(1, std::min(P.nslabs, cus));
        }
        return M2S_OK;
    }
    return M2S_ERR_UNSUPPORTED;
}

m2s_status check_ws(const m2s_stencil &A, const m2s_workspace *ws)
{
    if (!ws) return M2S_ERR_ARG;
    if (ws->kind != A.kind || ws->dtype != A.dtype || ws->g.nx != A.ext.nx ||
        ws->g.ny != A.ext.ny || ws->g.nz != A.ext.nz)
        return M2S_ERR_SHAPE;
    return M2S_OK;
}

// The tiled sweeps' tile table (27 points) and boundary store, laid out for
// nw compute wavefronts per tile; rebuilt (synchronously) when nw changes.
m2s_status ensure_tiles(m2s_workspace *ws, int nw)
{
    if (ws->bnd && ws->tile_nw == nw) return M2S_OK;
    if (ws->bnd || ws->tile_list) {
        if (hipDeviceSynchronize() != hipSuccess) return M2S_ERR_HIP;
        if (ws->bnd) (void)hipFree(ws->bnd);
        if (ws->tile_list) (void)hipFree(ws->tile_list);
        ws->bnd = nullptr;
        ws->tile_list = nullptr;
    }
    int64_t n = 1;
    size_t rb = 16;
    std::vector<int2> tiles;
    if (ws->kind == M2S_CONST27) {
        C27Layout L = c27_layout(ws->g, nw);
        n = std::max<int64_t>(L.bnd_elems, 1);
        rb = c27_record_bytes(ws->dtype);
        tiles.swap(L.tiles);
        ws->tile_ntiles = (int)tiles.size();
        ws->tile_nutb = L.nutb;
        ws->tile_ns = L.ns;
    } else if (ws->kind == M2S_VAR7) {
        const V7Layout L = v7_layout(ws->g, nw);
        n = std::max<int64_t>(L.bnd_elems, 1);
        rb = c27_record_bytes(ws->dtype);
        ws->tile_ntiles = L.ntiles;
        ws->tile_nutb = L.njt;
        ws->tile_ns = L.ns;
    } else {
        B7Layout L = b7_layout(ws->g, nw);
        n = std::max<int64_t>(L.bnd_elems, 1);
        tiles.swap(L.tiles);
        ws->tile_ntiles = L.ntiles;
        ws->tile_nutb = L.njt;
        ws->tile_ns = L.ns;
    }
    const size_t tb = sizeof(int2) * std::max<size_t>(tiles.size(), 1);
    // records start with epoch 0, which no launch uses
    if (hipMalloc(&ws->bnd, n * rb) != hipSuccess ||
        hipMalloc(&ws->tile_list, tb) != hipSuccess)
        return M2S_ERR_HIP;
    if ((!tiles.empty() &&
         hipMemcpy(ws->tile_list, tiles.data(), sizeof(int2) * tiles.size(),
                   hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemset(ws->bnd, 0, n * rb) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return M2S_ERR_HIP;
    ws->bnd_elems = n;
    ws->tile_nw = nw;
    return M2S_OK;
}

// One half-sweep out of place.
m2s_status half_sweep(const m2s_stencil &A, const Block7Consts *b7,
                      double omega, const void *r, const void *xin,
                      void *xout, bool bwd, bool zero_init,
                      m2s_workspace *ws, hipStream_t s)
{
    SweepPlan P{};
    m2s_status st = make_plan(A, P, true);
    if (st != M2S_OK) return st;
    if ((st = ensure_tiles(ws, P.slab_planes / 4)) != M2S_OK) return st;
    return hip_status(launch_sweep(A, b7, omega, r, xin, xout, bwd, zero_init,
                                   *ws, P, s));
}

// The FP32 27-point backward half-sweep from xin, its result stored widened
// to FP64 (the last sweep of a mixed-precision V-cycle).
m2s_status half_sweep_wide(const m2s_stencil &A, const void *r,
                           const void *xin, double *xout, m2s_workspace *ws,
                           hipStream_t s)
{
    SweepPlan P{};
    m2s_status st = make_plan(A, P, true);
    if (st != M2S_OK) return st;
    if ((st = ensure_tiles(ws, P.slab_planes / 4)) != M2S_OK) return st;
    return hip_status(launch_sweep27_wide(A, r, xin, xout, *ws, P, s));
}

}  // namespace

extern "C" {

const char *m2s_status_string(m2s_status s)
{
    switch (s) {
    case M2S_OK: return "ok";
    case M2S_ERR_ARG: return "invalid argument";
    case M2S_ERR_SHAPE: return "invalid or unsupported shape";
    case M2S_ERR_DTYPE: return "unsupported dtype";
    case M2S_ERR_ALIAS: return "input and output overlap";
    case M2S_ERR_HIP: return "HIP runtime error";
    case M2S_ERR_TIMEOUT: return "sweep dependency wait timed out";
    case M2S_ERR_BREAKDOWN: return "CG breakdown";
    case M2S_ERR_NOT_CONVERGED: return "CG did not converge";
    case M2S_ERR_UNSUPPORTED: return "operator kind not supported here";
    }
    return "unknown status";
}

// 2.0.0: m2s_ilu27_* renamed m2s_dilu27_*; m2s_ilu0_*, the PCG workspace
// entry points and m2s_stream added; 2.1.0: m2s_pcg_opts.check_every,
// m2s_ilu0_pack and m2s_ilu0_apply_packed
int m2s_version(void) { return 20100; }

m2s_status m2s_plan_sweep(const m2s_stencil *A, m2s_sweep_plan *plan)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (!plan) return M2S_ERR_ARG;
    SweepPlan P{};
    st = make_plan(*A, P, false);
    if (st != M2S_OK) return st;
    plan->slab_planes = P.slab_planes;
    plan->nslabs = P.nslabs;
    plan->row_slots = P.row_slots;
    plan->lag_row = P.lag_row;
    plan->lag_plane = P.lag_plane;
    if (A->kind == M2S_CONST27)  // u = j + k: T = i + 2u + 2k
        plan->steps = A->ext.nx + 2 * (P.row_slots - 1) +
                      2 * (P.slab_planes - 1);
    else  // VAR7, BLOCK7: T = i + j + k within a tile
        plan->steps = A->ext.nx + (P.row_slots - 1) + (P.slab_planes - 1);
    plan->threads = P.threads;
    plan->publish_every = P.publish_every;
    return M2S_OK;
}

m2s_status m2s_workspace_create(const m2s_stencil *A, m2s_workspace **out)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (!out) return M2S_ERR_ARG;
    *out = nullptr;
    m2s_workspace *ws = new (std::nothrow) m2s_workspace();
    if (!ws) return M2S_ERR_HIP;
    std::memset((Workspace *)ws, 0, sizeof(Workspace));
    ws->kind = A->kind;
    ws->dtype = A->dtype;
    ws->g = Grid{A->ext.nx, A->ext.ny, A->ext.nz};
    if (hipGetDevice(&ws->dev) != hipSuccess) { delete ws; return M2S_ERR_HIP; }
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    bool ok = hipMalloc(&ws->ticket, sizeof(uint64_t)) == hipSuccess &&
              hipMalloc(&ws->err, sizeof(int)) == hipSuccess &&
              hipMalloc(&ws->scratch, vb) == hipSuccess &&
              hipMalloc(&ws->scratch2, vb) == hipSuccess;
    if (ok) {
        SweepPlan P{};
        const m2s_status pst = make_plan(*A, P, false);
        if (pst != M2S_OK) {
            m2s_workspace_destroy(ws);
            return pst;
        }
        ok = ensure_tiles(ws, P.slab_planes / 4) == M2S_OK;
    }
    ok = ok && hipMemset(ws->ticket, 0, sizeof(uint64_t)) == hipSuccess &&
         hipMemset(ws->err, 0, sizeof(int)) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        m2s_workspace_destroy(ws);
        return M2S_ERR_HIP;
    }
    *out = ws;
    return M2S_OK;
}

void m2s_workspace_destroy(m2s_workspace *ws)
{
    if (!ws) return;
    (void)hipDeviceSynchronize();
    if (ws->ticket) (void)hipFree(ws->ticket);
    if (ws->err) (void)hipFree(ws->err);
    if (ws->scratch) (void)hipFree(ws->scratch);
    if (ws->scratch2) (void)hipFree(ws->scratch2);
    if (ws->bnd) (void)hipFree(ws->bnd);
    if (ws->tile_list) (void)hipFree(ws->tile_list);
    if (ws->b7c) (void)hipFree(ws->b7c);
    if (ws->xl_rec) (void)hipFree(ws->xl_rec);
    if (ws->ilb_doff) (void)hipFree(ws->ilb_doff);
    delete ws;
}

m2s_status m2s_check(m2s_workspace *ws, hipStream_t stream)
{
    if (!ws) return M2S_ERR_ARG;
    if (hipStreamSynchronize(stream) != hipSuccess) return M2S_ERR_HIP;
    int e = 0;
    if (hipMemcpy(&e, ws->err, sizeof(int), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return M2S_ERR_HIP;
    if (e) {
        // an aborted sweep leaves the ticket counter ahead of the host's
        // bookkeeping: resynchronise it before the workspace is reused
        uint64_t tk = 0;
        if (hipMemcpy(&tk, ws->ticket, sizeof(tk), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemset(ws->err, 0, sizeof(int)) != hipSuccess)
            return M2S_ERR_HIP;
        if (hipDeviceSynchronize() != hipSuccess) return M2S_ERR_HIP;
        ws->ticket_base = tk;
        return M2S_ERR_TIMEOUT;
    }
    return M2S_OK;
}

m2s_status m2s_spmv(const m2s_stencil *A, const void *x, void *y,
                    hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (!x || !y) return M2S_ERR_ARG;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(x, y, vb)) return M2S_ERR_ALIAS;
    return hip_status(launch_spmv(*A, x, y, stream));
}

m2s_status m2s_spmv_part(const m2s_stencil *A, int part, const void *x,
                         void *y, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!x || !y || (part != -1 && part != 1)) return M2S_ERR_ARG;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(x, y, vb)) return M2S_ERR_ALIAS;
    return hip_status(launch_spmv_part(*A, part, x, y, stream));
}

m2s_status m2s_symgs_oop(const m2s_stencil *A, const void *r,
                         const void *x_in, void *x_out, m2s_dir dir,
                         m2s_workspace *ws, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!r || !x_out) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD) return M2S_ERR_ARG;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(r, x_out, vb) || overlap(x_in, x_out, vb)) return M2S_ERR_ALIAS;
    return half_sweep(*A, nullptr, 1.0, r, x_in, x_out, dir == M2S_BWD,
                      x_in == nullptr, ws, stream);
}

m2s_status m2s_symgs(const m2s_stencil *A, const void *r, void *x,
                     m2s_dir dir, m2s_workspace *ws, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!r || !x) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(r, x, vb)) return M2S_ERR_ALIAS;
    if (dir == M2S_SYM) {
        if ((st = half_sweep(*A, nullptr, 1.0, r, x, ws->scratch, false,
                             false, ws, stream)) != M2S_OK)
            return st;
        return half_sweep(*A, nullptr, 1.0, r, ws->scratch, x, true, false,
                          ws, stream);
    }
    if ((st = half_sweep(*A, nullptr, 1.0, r, x, ws->scratch,
                         dir == M2S_BWD, false, ws, stream)) != M2S_OK)
        return st;
    return hip_status(launch_copy(x, ws->scratch, (int64_t)vb, stream));
}

m2s_status m2s_symgs_sequential(const m2s_stencil *A, const void *r, void *x,
                                m2s_dir dir, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (!r || !x) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(r, x, vb)) return M2S_ERR_ALIAS;
    if (dir & M2S_FWD)
        M2S_TRY(launch_sweep_sequential(*A, r, x, false, stream));
    if (dir & M2S_BWD)
        M2S_TRY(launch_sweep_sequential(*A, r, x, true, stream));
    return M2S_OK;
}

namespace {
// One 16-byte record per point (the x-line sweep; the band ILU(0) solves use
// a part), made on the first such call and zeroed: epoch 0 is never a
// launch's.
m2s_status ensure_point_records(m2s_workspace *ws, uint64_t rec_bytes,
                                hipStream_t stream)
{
    if (ws->xl_rec) return M2S_OK;
    void *rec = nullptr;
    if (hipMalloc(&rec, rec_bytes) != hipSuccess) return M2S_ERR_HIP;
    // kept only once cleared: a later call relies on the zero epochs
    if (hipMemsetAsync(rec, 0, rec_bytes, stream) != hipSuccess) {
        (void)hipFree(rec);
        return M2S_ERR_HIP;
    }
    ws->xl_rec = rec;
    return M2S_OK;
}
}  // namespace

m2s_status m2s_symgs_xline(const m2s_stencil *A, const void *r, void *x,
                           m2s_dir dir, m2s_workspace *ws, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_CONST27) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!r || !x) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    if (xline_lds_bytes(A->ext.nx) > 160 * 1024 - 64) return M2S_ERR_SHAPE;
    // records are addressed with 32-bit byte offsets
    const uint64_t rec_bytes = 16ull * (uint64_t)npoints(*A);
    if (rec_bytes >= (1ull << 32)) return M2S_ERR_SHAPE;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(r, x, vb)) return M2S_ERR_ALIAS;
    if ((st = ensure_point_records(ws, rec_bytes, stream)) != M2S_OK)
        return st;
    if (dir == M2S_SYM) {
        M2S_TRY(launch_xline_sweep(*A, r, x, ws->scratch, false, *ws,
                                   ws->xl_rec, stream));
        return hip_status(launch_xline_sweep(*A, r, ws->scratch, x, true, *ws,
                                             ws->xl_rec, stream));
    }
    M2S_TRY(launch_xline_sweep(*A, r, x, ws->scratch, dir == M2S_BWD, *ws,
                               ws->xl_rec, stream));
    return hip_status(launch_copy(x, ws->scratch, (int64_t)vb, stream));
}

m2s_status m2s_symgs_adjoint(const m2s_stencil *A, const void *g, void *gr,
                             void *gx, m2s_dir dir, m2s_workspace *ws,
                             hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!g || !gr || !gx) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(g, gr, vb) || overlap(g, gx, vb) || overlap(gr, gx, vb))
        return M2S_ERR_ALIAS;
    const m2s_dtype t = A->dtype;
    const int64_t n = npoints(*A);
    if (dir == M2S_FWD) {
        // gr = (D+U)^{-1} g: backward sweep from zero with right side g
        if ((st = half_sweep(*A, nullptr, 1.0, g, nullptr, gr, true, true, ws,
                             stream)) != M2S_OK)
            return st;
        M2S_TRY(launch_spmv_part(*A, -1, gr, gx, stream));
        return hip_status(launch_scale(gx, t, n, -1.0, stream));
    }
    if (dir == M2S_BWD) {
        if ((st = half_sweep(*A, nullptr, 1.0, g, nullptr, gr, false, true,
                             ws, stream)) != M2S_OK)
            return st;
        M2S_TRY(launch_spmv_part(*A, +1, gr, gx, stream));
        return hip_status(launch_scale(gx, t, n, -1.0, stream));
    }
    // SYM: x1 = F(r, x0), x2 = B(r, x1).  Reverse order:
    //   y2 = (D+L)^{-1} g ; g1 = -U y2 ; y1 = (D+U)^{-1} g1 ; gr = y2 + y1 ;
    //   gx0 = -L y1
    void *y2 = ws->scratch2;
    if ((st = half_sweep(*A, nullptr, 1.0, g, nullptr, y2, false, true, ws,
                         stream)) != M2S_OK)
        return st;
    M2S_TRY(launch_spmv_part(*A, +1, y2, gx, stream));
    M2S_TRY(launch_scale(gx, t, n, -1.0, stream));  // gx holds g1
    if ((st = half_sweep(*A, nullptr, 1.0, gx, nullptr, gr, true, true, ws,
                         stream)) != M2S_OK)
        return st;  // gr holds y1
    M2S_TRY(launch_spmv_part(*A, -1, gr, gx, stream));
    M2S_TRY(launch_scale(gx, t, n, -1.0, stream));
    // gr = y1 + y2
    return hip_status(launch_add(gr, y2, t, n, stream));
}

m2s_status m2s_ssor_sweep(const m2s_stencil *A, const void *b, void *x,
                          double omega, m2s_dir dir, m2s_workspace *ws,
                          hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!b || !x) return M2S_ERR_ARG;
    if (!(omega > 0.0 && omega < 2.0)) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(b, x, vb)) return M2S_ERR_ALIAS;
    Block7Consts C{};
    if (fill_block7_consts(A->blocks, C) != hipSuccess) return M2S_ERR_ARG;
    set_block7_omega(C, omega);
    if (dir == M2S_SYM) {
        if ((st = half_sweep(*A, &C, omega, b, x, ws->scratch, false, false,
                             ws, stream)) != M2S_OK)
            return st;
        return half_sweep(*A, &C, omega, b, ws->scratch, x, true, false, ws,
                          stream);
    }
    if ((st = half_sweep(*A, &C, omega, b, x, ws->scratch, dir == M2S_BWD,
                         false, ws, stream)) != M2S_OK)
        return st;
    return hip_status(launch_copy(x, ws->scratch, (int64_t)vb, stream));
}

m2s_status m2s_ssor_sweep_sequential(const m2s_stencil *A, const void *b,
                                     void *x, double omega, m2s_dir dir,
                                     hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (!b || !x) return M2S_ERR_ARG;
    if (!(omega > 0.0 && omega < 2.0)) return M2S_ERR_ARG;
    if (dir != M2S_FWD && dir != M2S_BWD && dir != M2S_SYM) return M2S_ERR_ARG;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(b, x, vb)) return M2S_ERR_ALIAS;
    Block7Consts C{};
    if (fill_block7_consts(A->blocks, C) != hipSuccess) return M2S_ERR_ARG;
    set_block7_omega(C, omega);
    if (dir & M2S_FWD)
        M2S_TRY(launch_sweep_sequential_b7(*A, C, omega, b, x, false, stream));
    if (dir & M2S_BWD)
        M2S_TRY(launch_sweep_sequential_b7(*A, C, omega, b, x, true, stream));
    return M2S_OK;
}

namespace {
m2s_status dilu27_prepare(const m2s_stencil *A, m2s_workspace *ws,
                         SweepPlan &P)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_CONST27) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    if ((st = make_plan(*A, P, true)) != M2S_OK) return st;
    return ensure_tiles(ws, P.slab_planes / 4);
}
}  // namespace

m2s_status m2s_dilu27_factor(const m2s_stencil *A, void *w, m2s_workspace *ws,
                            hipStream_t stream)
{
    if (!w) return M2S_ERR_ARG;
    SweepPlan P{};
    m2s_status st = dilu27_prepare(A, ws, P);
    if (st != M2S_OK) return st;
    return hip_status(launch_dilu27(*A, 1, nullptr, nullptr, w, *ws, P, stream));
}

m2s_status m2s_dilu27_apply(const m2s_stencil *A, const void *w,
                           const void *r, void *z, m2s_workspace *ws,
                           hipStream_t stream)
{
    if (!w || !r || !z) return M2S_ERR_ARG;
    SweepPlan P{};
    m2s_status st = dilu27_prepare(A, ws, P);
    if (st != M2S_OK) return st;
    const size_t vb = (size_t)npoints(*A) * elem_size(*A);
    if (overlap(w, r, vb) || overlap(w, z, vb) || overlap(r, z, vb))
        return M2S_ERR_ALIAS;
    M2S_TRY(launch_dilu27(*A, 2, r, w, ws->scratch, *ws, P, stream));
    return hip_status(launch_dilu27(*A, 3, ws->scratch, w, z, *ws, P, stream));
}

m2s_status m2s_ilu0_factor(const m2s_stencil *A, double *L, double *U,
                           hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_CONST27) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!L || !U) return M2S_ERR_ARG;
    const int64_t n = npoints(*A);
    if (overlap2(L, (size_t)(13 * n) * 8, U, (size_t)(14 * n) * 8))
        return M2S_ERR_ALIAS;
    return hip_status(launch_ilu0_factor(*A, L, U, stream));
}

m2s_status m2s_ilu0_apply(const m2s_stencil *A, const double *L,
                          const double *U, const double *r, double *z,
                          hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_CONST27) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!L || !U || !r || !z) return M2S_ERR_ARG;
    const int64_t n = npoints(*A);
    const size_t vb = 8 * (size_t)n;
    if (overlap(r, z, vb) || overlap2(L, (size_t)(13 * n) * 8, z, vb) ||
        overlap2(U, (size_t)(14 * n) * 8, z, vb))
        return M2S_ERR_ALIAS;
    return hip_status(launch_ilu0_apply(*A, L, U, r, z, stream));
}

namespace {
// checks shared by the packed ILU(0) entry points; the layout, its device
// offset table in the workspace
m2s_status ilb_prepare(const m2s_stencil *A, m2s_workspace *ws,
                       IlbLayout &L)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_CONST27) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if ((st = check_ws(*A, ws)) != M2S_OK) return st;
    const Grid g{A->ext.nx, A->ext.ny, A->ext.nz};
    L = ilb_layout(g);
    if (L.kt == 0) return M2S_ERR_UNSUPPORTED;   // ny > 512
    // packed arrays and records are addressed from 32-bit offsets
    if (14 * 8 * npoints(*A) >= ((int64_t)1 << 31) ||
        (int64_t)L.nbands * g.nx * g.ny * 16 >= ((int64_t)1 << 31) ||
        L.lds > 160 * 1024 - 64)
        return M2S_ERR_SHAPE;
    const int nd = (int)L.doff.size();
    if (ws->ilb_nd != nd || !ws->ilb_doff) {
        if (ws->ilb_doff) {
            if (hipDeviceSynchronize() != hipSuccess) return M2S_ERR_HIP;
            (void)hipFree(ws->ilb_doff);
            ws->ilb_doff = nullptr;
            ws->ilb_nd = 0;
        }
        int *d = nullptr;
        if (hipMalloc(&d, sizeof(int) * nd) != hipSuccess) return M2S_ERR_HIP;
        if (hipMemcpy(d, L.doff.data(), sizeof(int) * nd,
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return M2S_ERR_HIP;
        }
        ws->ilb_doff = d;
        ws->ilb_nd = nd;
    }
    return M2S_OK;
}
}  // namespace

m2s_status m2s_ilu0_pack(const m2s_stencil *A, const double *L,
                         const double *U, double *Lp, double *Up,
                         m2s_workspace *ws, hipStream_t stream)
{
    IlbLayout lay;
    m2s_status st = ilb_prepare(A, ws, lay);
    if (st != M2S_OK) return st;
    if (!L || !U || !Lp || !Up) return M2S_ERR_ARG;
    const int64_t n = npoints(*A);
    const size_t lb = (size_t)(13 * n) * 8, ub = (size_t)(14 * n) * 8;
    if (overlap2(Lp, lb, Up, ub) || overlap2(L, lb, Lp, lb) ||
        overlap2(L, lb, Up, ub) || overlap2(U, ub, Lp, lb) ||
        overlap2(U, ub, Up, ub))
        return M2S_ERR_ALIAS;
    return hip_status(launch_ilu0_pack(*A, ws->ilb_doff, L, U, Lp, Up, stream));
}

m2s_status m2s_ilu0_apply_packed(const m2s_stencil *A, const double *Lp,
                                 const double *Up, const double *r, double *z,
                                 m2s_workspace *ws, hipStream_t stream)
{
    IlbLayout lay;
    m2s_status st = ilb_prepare(A, ws, lay);
    if (st != M2S_OK) return st;
    if (!Lp || !Up || !r || !z) return M2S_ERR_ARG;
    const int64_t n = npoints(*A);
    const size_t vb = 8 * (size_t)n;
    if (overlap(r, z, vb) || overlap2(Lp, (size_t)(13 * n) * 8, z, vb) ||
        overlap2(Up, (size_t)(14 * n) * 8, z, vb))
        return M2S_ERR_ALIAS;
    if ((st = ensure_point_records(ws, 16ull * (uint64_t)n, stream)) !=
        M2S_OK)
        return st;
    const int64_t rec_elems =
        (int64_t)lay.nbands * A->ext.nx * A->ext.ny;
    return hip_status(launch_ilu0_apply_packed(
        *A, lay, ws->ilb_doff, Lp, Up, r, (double *)ws->scratch,
        (double *)ws->scratch2, z, *ws, ws->xl_rec, rec_elems, stream));
}

m2s_status m2s_penta_lines(int32_t nx, int32_t ny, int32_t nz, int32_t axis,
                           const double *coef, const double *r, double *x,
                           double *work, hipStream_t stream)
{
    if (!coef || !r || !x || !work || axis < 0 || axis > 2) return M2S_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 ||
        (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return M2S_ERR_SHAPE;
    const size_t vb = sizeof(double) * (size_t)nx * ny * nz;
    if (overlap2(coef, 5 * vb, r, vb) || overlap2(coef, 5 * vb, x, vb) ||
        overlap2(coef, 5 * vb, work, 2 * vb) || overlap(r, x, vb) ||
        overlap2(r, vb, work, 2 * vb) || overlap2(x, vb, work, 2 * vb))
        return M2S_ERR_ALIAS;
    return hip_status(
        launch_penta_lines(nx, ny, nz, axis, coef, r, x, work, stream));
}

m2s_status m2s_bt_lines(int32_t nx, int32_t ny, int32_t nz, int32_t axis,
                        const double *coef, const double *r, double *x,
                        double *work, hipStream_t stream)
{
    if (!coef || !r || !x || !work || axis < 0 || axis > 2) return M2S_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 ||
        (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return M2S_ERR_SHAPE;
    const size_t pb = sizeof(double) * (size_t)nx * ny * nz;  // per scalar
    if (overlap2(coef, 75 * pb, r, 5 * pb) || overlap2(coef, 75 * pb, x, 5 * pb) ||
        overlap2(coef, 75 * pb, work, 25 * pb) || overlap(r, x, 5 * pb) ||
        overlap2(r, 5 * pb, work, 25 * pb) || overlap2(x, 5 * pb, work, 25 * pb))
        return M2S_ERR_ALIAS;
    return hip_status(
        launch_bt_lines(nx, ny, nz, axis, coef, r, x, work, stream));
}

m2s_status m2s_jacobi9(int32_t nx, int32_t ny, double diag, double off,
                       const double *b, double *x, double *tmp, int32_t iters,
                       int32_t tblock, hipStream_t stream)
{
    if (!b || !x || !tmp || iters < 0 || !(diag != 0.0) ||
        !std::isfinite(diag) || !std::isfinite(off))
        return M2S_ERR_ARG;
    if (tblock != 1 && tblock != 2 && tblock != 4 && tblock != 8)
        return M2S_ERR_ARG;
    if (nx < 1 || ny < 1 || (int64_t)nx * ny >= ((int64_t)1 << 31))
        return M2S_ERR_SHAPE;
    const size_t vb = sizeof(double) * (size_t)nx * (size_t)ny;
    if (overlap(b, x, vb) || overlap(b, tmp, vb) || overlap(x, tmp, vb))
        return M2S_ERR_ALIAS;
    return hip_status(
        launch_jacobi9(nx, ny, diag, off, b, x, tmp, iters, tblock, stream));
}

m2s_status m2s_face_grad(const m2s_stencil *A, const double *u,
                         const double *lam, double *gkx, double *gky,
                         double *gkz, hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind != M2S_VAR7) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!u || !lam || !gkx || !gky || !gkz) return M2S_ERR_ARG;
    Grid g{A->ext.nx, A->ext.ny, A->ext.nz};
    return hip_status(launch_face_grad(g, u, lam, gkx, gky, gkz, stream));
}

m2s_status m2s_dot(const double *x, const double *y, int64_t n, double *out,
                   hipStream_t stream)
{
    if (!x || !y || !out || n < 0) return M2S_ERR_ARG;
    double *partials = nullptr;
    // a private partials buffer per call keeps concurrent callers apart
    if (hipMallocAsync((void **)&partials,
                       sizeof(double) * dot_partials_capacity(),
                       stream) != hipSuccess)
        return M2S_ERR_HIP;
    hipError_t e = hipMemsetAsync(partials, 0,
                                  sizeof(double) * dot_partials_capacity(),
                                  stream);
    if (e == hipSuccess) e = launch_dot(x, y, n, partials, out, stream);
    hipError_t f = hipFreeAsync(partials, stream);
    return (e == hipSuccess && f == hipSuccess) ? M2S_OK : M2S_ERR_HIP;
}

}  // extern "C"

// Reduction scratch of m2s_dot_noalloc: the per-block partial sums and the
// counter that launch_dot uses, as a file-scope device array (each GPU the
// library runs on holds its own copy from module load until the process
// ends).  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr int kDotScratchDoubles = 1032;
static __device__ __align__(256) double scratch[kDotScratchDoubles];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};

m2s_status dot_scratch(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return M2S_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return M2S_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess ||
            !p)
            return M2S_ERR_HIP;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return M2S_OK;
}
}  // namespace

extern "C" {

m2s_status m2s_dot_noalloc(const double *x, const double *y, int64_t n,
                           double *out, hipStream_t stream)
{
    if (!x || !y || !out || n < 0) return M2S_ERR_ARG;
    // the partials of launch_dot must fit the fixed scratch
    if (dot_partials_capacity() > kDotScratchDoubles)
        return M2S_ERR_UNSUPPORTED;
    double *sp = nullptr;
    m2s_status st = dot_scratch(&sp);
    if (st != M2S_OK) return st;
    // the scratch keeps the last call's contents: the counter starts at 0
    hipError_t e = launch_dot_reset(sp, stream);
    if (e == hipSuccess) e = launch_dot(x, y, n, sp, out, stream);
    return e == hipSuccess ? M2S_OK : M2S_ERR_HIP;
}

m2s_status m2s_stream(int32_t kind, const double *a, const double *b,
                      double *c, double s, int64_t n, hipStream_t stream)
{
    if (kind != 0 && kind != 1) return M2S_ERR_ARG;
    if (!a || !c || (kind == 1 && !b) || n < 0) return M2S_ERR_ARG;
    auto mis = [](const void *p) { return ((uintptr_t)p & 15) != 0; };
    if (mis(a) || mis(c) || (kind == 1 && mis(b))) return M2S_ERR_ARG;
    const size_t vb = 8 * (size_t)n;
    if (overlap(a, c, vb) || (kind == 1 && overlap(b, c, vb)))
        return M2S_ERR_ALIAS;
    if (n == 0) return M2S_OK;
    return hip_status(launch_stream(kind, a, b, c, s, n, stream));
}

m2s_status m2s_convert(const void *src, m2s_dtype src_t, void *dst,
                       m2s_dtype dst_t, int64_t n, hipStream_t stream)
{
    if (!src || !dst || n < 0) return M2S_ERR_ARG;
    if ((src_t != M2S_F64 && src_t != M2S_F32) ||
        (dst_t != M2S_F64 && dst_t != M2S_F32))
        return M2S_ERR_DTYPE;
    return hip_status(launch_convert(src, src_t, dst, dst_t, n, stream));
}

}  // extern "C"

// ------------------------------------------------------------------------
// Multigrid hierarchy and V-cycle.
// ------------------------------------------------------------------------
struct MgLevel {
    m2s_stencil A;        // this level's operator (dtype = hierarchy prec)
    void *kx = nullptr, *ky = nullptr, *kz = nullptr;  // owned (VAR7)
    void *r = nullptr;    // level right-hand side (levels >= 1)
    void *z = nullptr;    // level correction (levels >= 1)
    m2s_workspace *ws = nullptr;
};

struct m2s_mg {
    int levels;
    m2s_dtype prec;
    std::vector<MgLevel> L;
    void *r0 = nullptr, *z0 = nullptr;  // level-0 float buffers (F32 prec)
};

namespace {

// z_l = V-cycle(r_l) on level l.
// zwide (FP32 CONST27 levels only): the level's last sweep stores its
// result widened to FP64 there instead of into z.
m2s_status vcycle_level(m2s_mg *mg, int l, const void *r, void *z,
                        hipStream_t s, double *zwide = nullptr)
{
    MgLevel &lv = mg->L[l];
    m2s_status st;
    const bool coarsest = l == mg->levels - 1;
    auto last_bwd = [&]() -> m2s_status {
        if (zwide)
            return half_sweep_wide(lv.A, r, lv.ws->scratch, zwide, lv.ws, s);
        return half_sweep(lv.A, nullptr, 1.0, r, lv.ws->scratch, z, true,
                          false, lv.ws, s);
    };
    // z = 0 followed by one SymGS: the forward half starts from zero
    if ((st = half_sweep(lv.A, nullptr, 1.0, r, nullptr, lv.ws->scratch,
                         false, true, lv.ws, s)) != M2S_OK)
        return st;
    if (coarsest) return last_bwd();
    if ((st = half_sweep(lv.A, nullptr, 1.0, r, lv.ws->scratch, z, true,
                         false, lv.ws, s)) != M2S_OK)
        return st;
    MgLevel &cv = mg->L[l + 1];
    M2S_TRY(launch_restrict(lv.A, r, z, cv.r, s));
    if ((st = vcycle_level(mg, l + 1, cv.r, cv.z, s)) != M2S_OK) return st;
    M2S_TRY(launch_prolong(lv.A, cv.z, z, s));
    if ((st = half_sweep(lv.A, nullptr, 1.0, r, z, lv.ws->scratch, false,
                         false, lv.ws, s)) != M2S_OK)
        return st;
    return last_bwd();
}

}  // namespace

extern "C" {

void m2s_mg_destroy(m2s_mg *mg)
{
    if (!mg) return;
    (void)hipDeviceSynchronize();
    for (auto &lv : mg->L) {
        if (lv.kx) (void)hipFree(lv.kx);
        if (lv.ky) (void)hipFree(lv.ky);
        if (lv.kz) (void)hipFree(lv.kz);
        if (lv.r) (void)hipFree(lv.r);
        if (lv.z) (void)hipFree(lv.z);
        m2s_workspace_destroy(lv.ws);
    }
    if (mg->r0) (void)hipFree(mg->r0);
    if (mg->z0) (void)hipFree(mg->z0);
    delete mg;
}

m2s_status m2s_mg_create(const m2s_stencil *fine, int levels, m2s_dtype prec,
                         m2s_mg **out)
{
    m2s_status st = validate(fine);
    if (st != M2S_OK) return st;
    if (!out) return M2S_ERR_ARG;
    *out = nullptr;
    if (fine->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (fine->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (prec != M2S_F64 && prec != M2S_F32) return M2S_ERR_DTYPE;
    if (levels < 1 || levels > 12) return M2S_ERR_ARG;
    const int f = 1 << (levels - 1);
    if (fine->ext.nx % f || fine->ext.ny % f || fine->ext.nz % f)
        return M2S_ERR_SHAPE;
    m2s_mg *mg = new (std::nothrow) m2s_mg();
    if (!mg) return M2S_ERR_HIP;
    mg->levels = levels;
    mg->prec = prec;
    mg->L.resize(levels);
    const size_t es = prec == M2S_F64 ? 8 : 4;
    hipStream_t s = 0;
    for (int l = 0; l < levels; ++l) {
        MgLevel &lv = mg->L[l];
        lv.A = *fine;
        lv.A.dtype = prec;
        lv.A.ext = m2s_extent{fine->ext.nx >> l, fine->ext.ny >> l,
                              fine->ext.nz >> l};
        const int64_t n = npoints(lv.A);
        bool ok = true;
        if (fine->kind == M2S_VAR7) {
            Faces F{lv.A.ext.nx, lv.A.ext.ny, lv.A.ext.nz};
            ok = hipMalloc(&lv.kx, es * F.nfx()) == hipSuccess &&
                 hipMalloc(&lv.ky, es * F.nfy()) == hipSuccess &&
                 hipMalloc(&lv.kz, es * F.nfz()) == hipSuccess;
            if (ok && l == 0) {
                Faces F0{fine->ext.nx, fine->ext.ny, fine->ext.nz};
                ok = launch_convert(fine->kx, M2S_F64, lv.kx, prec, F0.nfx(),
                                    s) == hipSuccess &&
                     launch_convert(fine->ky, M2S_F64, lv.ky, prec, F0.nfy(),
                                    s) == hipSuccess &&
                     launch_convert(fine->kz, M2S_F64, lv.kz, prec, F0.nfz(),
                                    s) == hipSuccess;
            } else if (ok) {
                MgLevel &pv = mg->L[l - 1];
                Grid gf{pv.A.ext.nx, pv.A.ext.ny, pv.A.ext.nz};
                ok = launch_var7_coarsen(prec, gf, pv.kx, pv.ky, pv.kz, lv.kx,
                                         lv.ky, lv.kz, s) == hipSuccess;
            }
            lv.A.kx = lv.kx;
            lv.A.ky = lv.ky;
            lv.A.kz = lv.kz;
        }
        if (ok && l > 0)
            ok = hipMalloc(&lv.r, es * n) == hipSuccess &&
                 hipMalloc(&lv.z, es * n) == hipSuccess;
        if (ok) ok = m2s_workspace_create(&lv.A, &lv.ws) == M2S_OK;
        if (!ok) {
            m2s_mg_destroy(mg);
            return M2S_ERR_HIP;
        }
    }
    if (prec == M2S_F32) {
        const int64_t n = npoints(*fine);
        if (hipMalloc(&mg->r0, 4 * n) != hipSuccess ||
            hipMalloc(&mg->z0, 4 * n) != hipSuccess) {
            m2s_mg_destroy(mg);
            return M2S_ERR_HIP;
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        m2s_mg_destroy(mg);
        return M2S_ERR_HIP;
    }
    *out = mg;
    return M2S_OK;
}

m2s_status m2s_mg_vcycle(m2s_mg *mg, const double *r, double *z,
                         hipStream_t stream)
{
    if (!mg || !r || !z) return M2S_ERR_ARG;
    const int64_t n = npoints(mg->L[0].A);
    if (overlap(r, z, 8 * (size_t)n)) return M2S_ERR_ALIAS;
    if (mg->prec == M2S_F64) return vcycle_level(mg, 0, r, z, stream);
    M2S_TRY(launch_convert(r, M2S_F64, mg->r0, M2S_F32, n, stream));
    // the 27-point kernel's last sweep writes the FP64 z itself (its
    // widened output uses 32-bit byte offsets); otherwise a conversion pass
    const bool wide = mg->L[0].A.kind == M2S_CONST27 &&
                      n * 8 < ((int64_t)1 << 31);
    m2s_status st =
        vcycle_level(mg, 0, mg->r0, mg->z0, stream, wide ? z : nullptr);
    if (st != M2S_OK || wide) return st;
    return hip_status(launch_convert(mg->z0, M2S_F32, z, M2S_F64, n, stream));
}

}  // extern "C"

// ------------------------------------------------------------------------
// PCG.
// ------------------------------------------------------------------------
namespace {

}  // namespace

// The PCG vectors and scalars of one operator, made once and reused by
// every solve (m2s_pcg_solve_ws), so that a solve allocates nothing.
struct m2s_pcg_workspace {
    m2s_kind kind;
    m2s_extent ext;
    double *r = nullptr, *z = nullptr, *p = nullptr, *ap = nullptr;
    double *sc = nullptr, *partials = nullptr;
    m2s_workspace *ws = nullptr;  // sweeps of the SYMGS preconditioner
};

namespace {

m2s_status workspace_error(m2s_workspace *ws)
{
    if (!ws) return M2S_OK;
    int e = 0;
    if (hipMemcpy(&e, ws->err, sizeof(int), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return M2S_ERR_HIP;
    if (e) {
        uint64_t tk = 0;
        (void)hipMemcpy(&tk, ws->ticket, sizeof(tk), hipMemcpyDeviceToHost);
        (void)hipMemset(ws->err, 0, sizeof(int));
        (void)hipDeviceSynchronize();
        ws->ticket_base = tk;
        return M2S_ERR_TIMEOUT;
    }
    return M2S_OK;
}

m2s_status mg_error(m2s_mg *mg)
{
    if (!mg) return M2S_OK;
    for (auto &lv : mg->L) {
        m2s_status st = workspace_error(lv.ws);
        if (st != M2S_OK) return st;
    }
    return M2S_OK;
}

}  // namespace

extern "C" m2s_status m2s_pcg_solve_ws(const m2s_stencil *A,
                                       m2s_precond precond, m2s_mg *mg,
                                       const double *b, double *x,
                                       const m2s_pcg_opts *opts,
                                       m2s_pcg_info *info, double *hist,
                                       m2s_pcg_workspace *W,
                                       hipStream_t stream)
{
    auto t0 = std::chrono::steady_clock::now();
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!b || !x || !opts) return M2S_ERR_ARG;
    if (opts->max_iter < 0) return M2S_ERR_ARG;
    if (precond != M2S_PC_NONE && precond != M2S_PC_SYMGS &&
        precond != M2S_PC_MG)
        return M2S_ERR_ARG;
    if (precond == M2S_PC_MG) {
        if (!mg) return M2S_ERR_ARG;
        const m2s_extent &e = mg->L[0].A.ext;
        if (e.nx != A->ext.nx || e.ny != A->ext.ny || e.nz != A->ext.nz ||
            mg->L[0].A.kind != A->kind)
            return M2S_ERR_SHAPE;
    }
    if (!W) return M2S_ERR_ARG;
    if (W->kind != A->kind || W->ext.nx != A->ext.nx ||
        W->ext.ny != A->ext.ny || W->ext.nz != A->ext.nz)
        return M2S_ERR_SHAPE;
    const int64_t n = npoints(*A);
    const size_t vb = 8 * (size_t)n;
    if (overlap(b, x, vb)) return M2S_ERR_ALIAS;
    // b and x must not be one of the workspace's own vectors
    for (const double *v : {W->r, W->z, W->p, W->ap})
        if (overlap(b, v, vb) || overlap(x, v, vb)) return M2S_ERR_ALIAS;
    m2s_pcg_workspace &B = *W;
    // the scalars start at zero (the partials' counter re-arms itself)
    M2S_TRY(hipMemsetAsync(B.sc, 0, sizeof(double) * SC_N, stream));
    double hsc[SC_N];
    auto fetch = [&]() -> m2s_status {
        if (hipMemcpyAsync(hsc, B.sc, sizeof(hsc), hipMemcpyDeviceToHost,
                           stream) != hipSuccess)
            return M2S_ERR_HIP;
        if (hipStreamSynchronize(stream) != hipSuccess) return M2S_ERR_HIP;
        return M2S_OK;
    };
    auto true_residual = [&]() -> m2s_status {
        M2S_TRY(launch_spmv(*A, x, B.ap, stream));
        M2S_TRY(launch_residual(b, B.ap, B.r, n, B.partials, B.sc + SC_RR,
                                stream));
        return M2S_OK;
    };
    if ((st = true_residual()) != M2S_OK) return st;
    if ((st = fetch()) != M2S_OK) return st;
    const double normr0 = std::sqrt(hsc[SC_RR]);
    double normr = normr0;
    m2s_status result = M2S_ERR_NOT_CONVERGED;
    const bool lazy = opts->rtol <= 0 && opts->replace_every <= 0 && !hist;
    const int check_every = std::max(1, opts->check_every);
    int it = 0;
    if (hist) hist[0] = 1.0;
    if (!std::isfinite(normr0)) result = M2S_ERR_BREAKDOWN;
    else if (normr0 == 0.0) result = M2S_OK;
    else {
        for (it = 1; it <= opts->max_iter; ++it) {
            const double *zz = B.z;
            if (precond == M2S_PC_NONE) {
                zz = B.r;
            } else if (precond == M2S_PC_SYMGS) {
                if ((st = half_sweep(*A, nullptr, 1.0, B.r, nullptr,
                                     B.ws->scratch, false, true, B.ws,
                                     stream)) != M2S_OK)
                    return st;
                if ((st = half_sweep(*A, nullptr, 1.0, B.r, B.ws->scratch,
                                     B.z, true, false, B.ws, stream)) !=
                    M2S_OK)
                    return st;
            } else {
                if ((st = m2s_mg_vcycle(mg, B.r, B.z, stream)) != M2S_OK)
                    return st;
            }
            M2S_TRY(hipMemcpyAsync(B.sc + SC_RZ_OLD, B.sc + SC_RZ,
                                   sizeof(double), hipMemcpyDeviceToDevice,
                                   stream));
            M2S_TRY(launch_dot(B.r, zz, n, B.partials, B.sc + SC_RZ, stream));
            M2S_TRY(launch_update_p(zz, B.p, n, B.sc, it == 1, stream));
            M2S_TRY(launch_spmv_dot(*A, B.p, B.ap, B.partials, B.sc + SC_PAP,
                                    stream));
            M2S_TRY(launch_update_xr(x, B.r, B.p, B.ap, n, B.sc, B.partials,
                                     it, stream));
            // a fixed-iteration run without history or replacement has no
            // test to make before its last iteration, and a convergence
            // test runs only every check_every iterations: in between the
            // scalars stay on the device (a breakdown is latched there) and
            // the host does not wait for each iteration
            if (lazy && it < opts->max_iter) continue;
            const bool replace_now =
                opts->replace_every > 0 && it % opts->replace_every == 0;
            if (!hist && !replace_now && it < opts->max_iter &&
                it % check_every != 0)
                continue;
            if ((st = fetch()) != M2S_OK) return st;
            const double pap = hsc[SC_PAP];
            normr = std::sqrt(hsc[SC_RR]);
            if (hsc[SC_BD] != 0.0 || !(pap > 0.0) || !std::isfinite(pap) ||
                !std::isfinite(normr) || !std::isfinite(hsc[SC_RZ])) {
                // the update kernels leave x, r and p alone from the
                // iteration that latched the breakdown on
                if (hsc[SC_BD] != 0.0) it = (int)hsc[SC_BDIT];
                result = M2S_ERR_BREAKDOWN;
                break;
            }
            const bool replace =
                opts->replace_every > 0 && it % opts->replace_every == 0;
            const bool check = opts->rtol > 0 && normr / normr0 <= opts->rtol;
            if (replace || check) {
                if ((st = true_residual()) != M2S_OK) return st;
                if ((st = fetch()) != M2S_OK) return st;
                normr = std::sqrt(hsc[SC_RR]);
            }
            if (hist) hist[it] = normr / normr0;
            if (opts->rtol > 0 && normr / normr0 <= opts->rtol) {
                result = M2S_OK;
                break;
            }
        }
        if (it > opts->max_iter) {
            it = opts->max_iter;
            if (opts->rtol <= 0) result = M2S_OK;
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return M2S_ERR_HIP;
    m2s_status werr = precond == M2S_PC_MG ? mg_error(mg)
                                           : workspace_error(B.ws);
    if (werr != M2S_OK) result = werr;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        // true residual of the returned x
        if (true_residual() == M2S_OK && fetch() == M2S_OK)
            info->true_rel_res =
                normr0 > 0 ? std::sqrt(hsc[SC_RR]) / normr0 : 0.0;
        info->iters = it;
        info->rel_res = normr0 > 0 ? normr / normr0 : 0.0;
        info->r0_norm = normr0;
        info->status = result;
        info->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    return result;
}

extern "C" m2s_status m2s_pcg_workspace_create(const m2s_stencil *A,
                                               m2s_pcg_workspace **out)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (!out) return M2S_ERR_ARG;
    *out = nullptr;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    m2s_pcg_workspace *W = new (std::nothrow) m2s_pcg_workspace();
    if (!W) return M2S_ERR_HIP;
    W->kind = A->kind;
    W->ext = A->ext;
    const size_t vb = 8 * (size_t)npoints(*A);
    const size_t pb = sizeof(double) * dot_partials_capacity();
    bool ok = hipMalloc((void **)&W->r, vb) == hipSuccess &&
              hipMalloc((void **)&W->z, vb) == hipSuccess &&
              hipMalloc((void **)&W->p, vb) == hipSuccess &&
              hipMalloc((void **)&W->ap, vb) == hipSuccess &&
              hipMalloc((void **)&W->sc, sizeof(double) * SC_N) ==
                  hipSuccess &&
              hipMalloc((void **)&W->partials, pb) == hipSuccess &&
              hipMemset(W->partials, 0, pb) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    if (ok) ok = m2s_workspace_create(A, &W->ws) == M2S_OK;
    if (!ok) {
        m2s_pcg_workspace_destroy(W);
        return M2S_ERR_HIP;
    }
    *out = W;
    return M2S_OK;
}

extern "C" void m2s_pcg_workspace_destroy(m2s_pcg_workspace *W)
{
    if (!W) return;
    (void)hipDeviceSynchronize();
    for (double *v : {W->r, W->z, W->p, W->ap, W->sc, W->partials})
        if (v) (void)hipFree(v);
    if (W->ws) m2s_workspace_destroy(W->ws);
    delete W;
}

extern "C" m2s_status m2s_pcg_solve(const m2s_stencil *A,
                                    m2s_precond precond, m2s_mg *mg,
                                    const double *b, double *x,
                                    const m2s_pcg_opts *opts,
                                    m2s_pcg_info *info, double *hist,
                                    hipStream_t stream)
{
    m2s_status st = validate(A);
    if (st != M2S_OK) return st;
    if (A->kind == M2S_BLOCK7_5) return M2S_ERR_UNSUPPORTED;
    if (A->dtype != M2S_F64) return M2S_ERR_DTYPE;
    if (!b || !x || !opts) return M2S_ERR_ARG;
    m2s_pcg_workspace *W = nullptr;
    if ((st = m2s_pcg_workspace_create(A, &W)) != M2S_OK) return st;
    st = m2s_pcg_solve_ws(A, precond, mg, b, x, opts, info, hist, W, stream);
    m2s_pcg_workspace_destroy(W);
    return st;
}
