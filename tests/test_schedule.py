"""CPU checks of the wavefront schedule (no GPU): the hyperplane legality
criterion of Sec. 6.1.3 (pinned to the paper's 2-D example), and a brute-
force model of the slab/row-slot schedule that libm2s.so plans
(m2s_plan_sweep), checking that every dependence of the lexicographic sweep
is satisfied by it."""
import itertools
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def phi_coeffs(partition_sizes):
    """Eq. (hyperplane): phi(x) = sum_i (prod_{j>i} N^t_j) x_i."""
    n = len(partition_sizes) + 1
    c = []
    for i in range(n):
        prod = 1
        for s in partition_sizes[i:]:
            prod *= s
        c.append(prod)
    return c


def legal(coeffs, offsets):
    return all(np.dot(coeffs, d) > 0 for d in offsets)


def test_paper_2d_example():
    with open(os.path.join(GOLD, "paper_sec6_hyperplane_2d.json")) as fh:
        g = json.load(fh)
    c = phi_coeffs(g["partition_sizes"])
    assert c == g["phi_coefficients"]
    assert legal(c, g["legal_offsets_b_minus_a"])
    assert not legal(c, g["legal_offsets_b_minus_a"] +
                     [g["illegal_offset_b_minus_a"]])


def lower_offsets_27():
    """b - a for a lower neighbour a of b, in (dk, dj, di) order."""
    out = []
    for dk, dj, di in itertools.product((-1, 0, 1), repeat=3):
        if (dk, dj, di) < (0, 0, 0):
            out.append((-dk, -dj, -di))
    return out


def lower_offsets_7():
    return [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_27_point_hyperplane_weights():
    # (k, j, i) weights (4, 2, 1) are legal and minimal; (2, 1, 1) is not.
    assert len(lower_offsets_27()) == 13
    assert legal((4, 2, 1), lower_offsets_27())
    assert not legal((2, 1, 1), lower_offsets_27())
    assert not legal((3, 2, 1), lower_offsets_27())
    assert legal((1, 1, 1), lower_offsets_7())


# ---------------------------------------------------------------------------
# Model of the GPU schedule (mirrors the sweep kernel's index arithmetic).
# ---------------------------------------------------------------------------
def model_schedule(shape, plan, c27):
    nz, ny, nx = shape
    Bk, R = plan["slab_planes"], plan["row_slots"]
    LJ, LK = plan["lag_row"], plan["lag_plane"]
    hx = hy = 1 if c27 else 0
    D = 1 + hx + LJ * hy + LK * (Bk - 1)
    G = plan["publish_every"]
    step = np.empty(shape, dtype=np.int64)
    slab = np.empty(shape, dtype=np.int64)
    owner = {}
    for k in range(nz):
        K, kk = divmod(k, Bk)
        for j in range(ny):
            s = j % R
            for i in range(nx):
                t = i + LJ * j + LK * kk
                # the kernel's inverse mapping must give back (i, j)
                rel = t - LK * kk - LJ * s
                m = 0 if R >= ny else rel // (LJ * R)
                assert (rel - m * LJ * R, s + m * R) == (i, j)
                key = (K, kk, s, t)
                assert key not in owner, "two points on one thread and step"
                owner[key] = (i, j, k)
                step[k, j, i] = t
                slab[k, j, i] = K
    Tfull = nx + LJ * (ny - 1) + LK * (Bk - 1)
    return step, slab, D, G, Tfull


@pytest.mark.parametrize("kind,shape", [
    ("c27", (9, 7, 6)), ("c27", (5, 3, 11)), ("c27", (16, 16, 16)),
    ("c27", (13, 26, 9)), ("v7", (9, 7, 6)), ("v7", (6, 5, 12)),
    ("b7", (7, 4, 5)),
])
@pytest.mark.parametrize("bk", [1, 2, 3, 0])
def test_gpu_schedule_satisfies_all_dependences(kind, shape, bk, monkeypatch):
    import paper_2204_13304_amd as m
    if bk:
        monkeypatch.setenv("M2S_SLAB_PLANES", str(bk))
    nz, ny, nx = shape
    if kind == "c27":
        A = m.const27(shape)
    elif kind == "v7":
        import torch
        A = m.Stencil.__new__(m.Stencil)
        A.kind, A.shape, A.dtype = 1, shape, torch.float64
        A.diag = A.off = 0.0
        A.blocks = None
        # faces are only read by the kernels; planning needs non-null
        # pointers, so fake addresses are enough for this host-only call
        import ctypes as C
        from paper_2204_13304_amd import _lib as L
        s = L.StencilC()
        s.kind, s.dtype = 1, 0
        s.ext = L.Extent(nx, ny, nz)
        s.kx = s.ky = s.kz = 8
        A._c = s
    else:
        A = m.block7(shape, np.eye(5)[None].repeat(7, 0) * 10)
    plan = m.plan_sweep(A)
    c27 = kind == "c27"
    step, slab, D, G, Tfull = model_schedule(shape, plan, c27)
    offs = lower_offsets_27() if c27 else lower_offsets_7()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                t, K = step[k, j, i], slab[k, j, i]
                for dk, dj, di in offs:
                    a = (k - dk, j - dj, i - di)
                    if not (0 <= a[0] < nz and 0 <= a[1] < ny and
                            0 <= a[2] < nx):
                        continue
                    ta, Ka = step[a], slab[a]
                    if Ka == K:
                        assert ta < t, (a, (k, j, i))
                    elif c27:
                        # the 27-point kernel hands the previous slab's top
                        # plane over value by value: row j' of plane k0-1 is
                        # staged at column i' one step before its first read
                        # (at local step i' + 2j' - 3, by row j'-1) and the
                        # stage waits until the value has been written
                        assert Ka == K - 1
                        _, jp, ip = a
                        stage_step = ip - 4 + 2 * jp
                        first_read = ip + 2 * jp - 3
                        assert stage_step < first_read <= t
                    else:
                        # producer slab must be exactly the previous one and
                        # covered by the progress wait of the G-window
                        assert Ka == K - 1
                        t0 = t - t % G
                        need = min(Tfull, t0 + G - 1 + D)
                        assert ta < need, (a, (k, j, i), ta, need)
