"""CPU checks of the wavefront schedule (no GPU): the hyperplane legality
criterion of Sec. 6.1.3 (pinned to the paper's 2-D example), and models of
the three tiled sweep kernels (27-point, VAR7, block SSOR) that replay each
kernel's index arithmetic step by step on symbolic values, checking that
every read of the lexicographic sweep sees the right value, that no two
wavefronts race on a slot, and that the tilings match what libm2s.so plans
(m2s_plan_sweep); and a model of the tiles' hand-off protocol (tickets in
dependency order, epoch-tagged records, bounded waits) with fault
injection: a withheld record must end in a latched time-out, not a hang."""
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


def _fake_var7(m, shape):
    """A VAR7 stencil descriptor for host-only planning calls: faces are
    only read by the kernels and planning needs non-null pointers, so fake
    addresses are enough."""
    import torch
    from paper_2204_13304_amd import _lib as L
    nz, ny, nx = shape
    A = m.Stencil.__new__(m.Stencil)
    A.kind, A.shape, A.dtype = 1, shape, torch.float64
    A.diag = A.off = 0.0
    A.blocks = None
    s = L.StencilC()
    s.kind, s.dtype = 1, 0
    s.ext = L.Extent(nx, ny, nz)
    s.kx = s.ky = s.kz = 8
    A._c = s
    return A


# ---------------------------------------------------------------------------
# Model of the tiled 27-point sweep kernel.  It replays the kernel's index
# arithmetic (tiles of 16 u = j + k by KT planes, LDS rings of 32 x columns
# and 16 r columns, the five per-step roles of every lane) on symbolic
# values and checks every read: lower neighbours must hold the new value,
# upper ones the old value, anything outside the grid zero; no slot may be
# written by one wavefront and touched by another in the same step; and
# every point must be stored exactly once, with its new value.
# ---------------------------------------------------------------------------
TU, RU, W, WR, PRE = 16, 20, 32, 16, 18


def c27_tile_list(shape, kt):
    nz, ny, nx = shape
    out = []
    for vt in range(-(-nz // kt)):
        k0, kmax = kt * vt, min(kt * vt + kt, nz) - 1
        for ut in range(k0 // TU, (kmax + ny - 1) // TU + 1):
            ulo, uhi = TU * ut, TU * ut + TU - 1
            if max(k0, ulo - ny + 1) <= min(kmax, uhi):
                out.append((ut, vt))
    return out


def simulate_c27_tiles(shape, nw, zero_start=False, POLL=3):
    """Wavefronts 0 .. nw-1 compute (one lane per row), nw .. 2nw-1 memory
    (wavefront nw + m stages x_old / r of compute wavefront m's rows and
    stores its pieces), 2nw polls the neighbour tiles' boundary records."""
    nz, ny, nx = shape
    KT = 4 * nw
    tiles = c27_tile_list(shape, KT)
    ticket = {t: n for n, t in enumerate(tiles)}
    stored = {}

    def valid(u, k):
        return 0 <= u - k < ny and 0 <= k < nz

    def old(u, k, c):
        if not valid(u, k) or not 0 <= c < nx or zero_start:
            return 0
        return ("old", u - k, k, c)

    def xslot(kq, uq, c):
        return ((kq + 1) * RU + (uq + 2), c % W)

    for (ut, vt) in tiles:
        u0, k0 = TU * ut, KT * vt
        T0 = 2 * (u0 + k0)
        xr, rr = {}, {}
        T_start = T0 - 6 - PRE
        T_lastc = T0 + 2 * (TU - 1) + 2 * (KT - 1) + nx - 1
        nblk = (T_lastc + 9 - T_start + 15) // 16
        for blk in range(nblk):
            for ph in range(16):
                T = T_start + 16 * blk + ph
                writes = []      # (ring, slot, value, wave)
                reads = []       # (ring, slot, wave, expected)
                for m in range(nw):
                    wm = nw + m
                    for lane in range(64):
                        q8, r8, p8 = lane & 7, lane >> 3, ph & 7
                        # 8 rows per step: x_old window [f + 8, f + 16),
                        # r window [f + 1, f + 9), store [f - 8, f)
                        rho = 8 * p8 + r8
                        uL, kL = rho & 15, 4 * m + (rho >> 4)
                        u, k = u0 + uL, k0 + kL
                        f = T - 2 * (u + k)
                        cx, cr, cs = f + 9 + q8, f + 1 + q8, f - 8 + q8
                        vx = 0 if T - 8 < T_start else old(u, k, cx)
                        writes.append(("x", xslot(kL, uL, cx), vx, wm))
                        vr = (0 if T - 8 < T_start or not valid(u, k) or
                              not 0 <= cr < nx else ("r", u - k, k, cr))
                        writes.append(("r", (kL * TU + uL, cr % WR), vr, wm))
                        if valid(u, k) and 0 <= cs < nx:
                            reads.append(("x", xslot(kL, uL, cs), wm,
                                          ("new", u - k, k, cs)))
                            key = (k, u - k, cs)
                            assert key not in stored, key
                            stored[key] = True
                        # old-value halo rows
                        if p8 < 4:
                            h = 8 * p8 + r8
                            lo = h < 8
                            if lo or (m == nw - 1 and h < 26):
                                uH = 16 + (h & 1) if lo else h - 8
                                kH = 4 * m + (h >> 1) if lo else KT
                                cxh = T - 2 * (u0 + uH + k0 + kH) + 9 + q8
                                vh = (0 if T - 8 < T_start else
                                      old(u0 + uH, k0 + kH, cxh))
                                writes.append(("x", xslot(kH, uH, cxh), vh,
                                               wm))
                # poll wavefront
                wp = 2 * nw
                for lane in range(2 * KT + 18):
                    if lane < 2 * KT:
                        hu, hk = -2 + (lane & 1), lane >> 1
                        prod, hidx = (ut - 1, vt), lane
                    elif lane < 2 * KT + 14:
                        hu, hk = lane - 2 * KT, -1
                        prod, hidx = (ut, vt - 1), 2 * KT + hu
                    elif lane < 2 * KT + 16:
                        hu, hk = 14 + lane - 2 * KT - 14, -1
                        prod = (ut, vt - 1)
                        hidx = 2 * (KT - 1) + hu - 14
                    else:
                        hu, hk = -2 + lane - 2 * KT - 16, -1
                        prod = (ut - 1, vt - 1)
                        hidx = 2 * (KT - 1) + hu + 2
                    hug, hkg = u0 + hu, k0 + hk
                    c = T - 2 * (hug + hkg)
                    if valid(hug, hkg) and c >= 0:
                        if c < nx:
                            # the record was polled POLL steps earlier
                            assert T - POLL >= T_start, (T, T_start)
                            assert prod in ticket and \
                                ticket[prod] < ticket[(ut, vt)]
                            # the producer publishes this row at entry hidx
                            uup = hug - TU * prod[0]
                            kkp = hkg - KT * prod[1]
                            assert 0 <= uup < TU and 0 <= kkp < KT
                            ent = ((uup - 14) + 2 * kkp if uup >= 14 else
                                   (2 * KT + uup if kkp == KT - 1 else -1))
                            assert ent == hidx, (ent, hidx)
                            v = ("new", hug - hkg, hkg, c)
                        else:
                            v = 0
                        writes.append(("x", xslot(hk, hu, c), v, wp))
                # compute wavefronts
                for w in range(nw):
                    for lane in range(64):
                        sub, cl = lane >> 4, lane & 15
                        kk = 4 * w + sub
                        u, k = u0 + cl, k0 + kk
                        f = T - 2 * (u + k)
                        # v2 (u, k-1) and v3 (u-1, k) of column f + 1 are
                        # read last; the other six rows and the own old
                        # value are read for column f + 2
                        for du, dk, c in ((0, -1, f + 1), (-1, 0, f + 1),
                                          (-2, -1, f + 2), (-1, -1, f + 2),
                                          (1, 0, f + 2), (0, 1, f + 2),
                                          (1, 1, f + 2), (2, 1, f + 2)):
                            if not (valid(u, k) and -1 <= c <= nx):
                                continue
                            ua, ka = u + du, k + dk
                            lower = dk < 0 or (dk == 0 and du < 0)
                            if not valid(ua, ka) or not 0 <= c < nx:
                                e = 0
                            elif lower:
                                e = ("new", ua - ka, ka, c)
                            else:
                                e = old(ua, ka, c)
                            reads.append(("x", xslot(kk + dk, cl + du, c), w,
                                          e))
                        c = f + 2
                        if valid(u, k) and -1 <= c <= nx:
                            reads.append(("x", xslot(kk, cl, c), w,
                                          old(u, k, c) if c < nx else 0))
                        if valid(u, k) and 0 <= f < nx:
                            reads.append(("r", (kk * TU + cl, f % WR), w,
                                          ("r", u - k, k, f)))
                            writes.append(("x", xslot(kk, cl, f),
                                           ("new", u - k, k, f), w))
                # one step: no slot is touched by two wavefronts if one of
                # them writes it; reads see the previous step's state
                wsl = {}
                for ring, slot, v, w in writes:
                    prev = wsl.get((ring, slot))
                    assert prev is None or prev[1] == w, \
                        ("write race", ring, slot, T)
                    wsl[(ring, slot)] = (v, w)
                for ring, slot, w, e in reads:
                    assert (ring, slot) not in wsl, \
                        ("read/write race", ring, slot, T, w, wsl[(ring, slot)])
                    mem = xr if ring == "x" else rr
                    got = mem.get(slot, 0)
                    assert got == e, (T, ring, slot, got, e)
                for (ring, slot), (v, w) in wsl.items():
                    (xr if ring == "x" else rr)[slot] = v
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                assert (k, j, i) in stored, ("not stored", (k, j, i))


@pytest.mark.parametrize("shape", [(9, 7, 6), (5, 3, 11), (6, 20, 37),
                                   (13, 5, 4), (17, 18, 3), (1, 1, 1)])
@pytest.mark.parametrize("nw", [1, 2, 4])
def test_c27_tile_model(shape, nw):
    # the kernel polls the boundary records 3 steps ahead
    simulate_c27_tiles(shape, nw)


def test_c27_tile_model_zero_start():
    simulate_c27_tiles((6, 9, 5), 2, zero_start=True)


def test_c27_tile_dependences_point_to_earlier_tiles():
    # every lower neighbour lies in the same tile or in tile (u-1, k),
    # (u, k-1) or (u-1, k-1), each with an earlier ticket
    for shape, kt in (((9, 7, 6), 4), ((23, 40, 5), 8), ((16, 16, 16), 16)):
        nz, ny, nx = shape
        tiles = c27_tile_list(shape, kt)
        ticket = {t: n for n, t in enumerate(tiles)}
        for k in range(nz):
            for j in range(ny):
                u = j + k
                tp = (u // TU, k // kt)
                assert tp in ticket
                for dk, dj, di in lower_offsets_27():
                    ka, ja = k - dk, j - dj
                    if not (0 <= ka < nz and 0 <= ja < ny):
                        continue
                    ta = ((ja + ka) // TU, ka // kt)
                    assert ta in (tp, (tp[0] - 1, tp[1]), (tp[0], tp[1] - 1),
                                  (tp[0] - 1, tp[1] - 1))
                    assert ticket[ta] <= ticket[tp]


@pytest.mark.parametrize("shape", [(9, 7, 6), (16, 16, 16), (13, 26, 9)])
def test_c27_plan_matches_tile_model(shape, monkeypatch):
    import paper_2204_13304_amd as m
    for nw in (1, 2, 4):
        monkeypatch.setenv("M2S_C27_WAVES", str(nw))
        p = m.plan_sweep(m.const27(shape))
        assert p["slab_planes"] == 4 * nw
        # nw compute + nw memory wavefronts + 1 poll wavefront
        assert p["threads"] == 64 * (2 * nw + 1)
        assert p["nslabs"] == len(c27_tile_list(shape, 4 * nw))


# ---------------------------------------------------------------------------
# Model of the tiled block-SSOR sweep kernel (7-point, 5 components): tiles
# of 16 j by 4 k, seven roles -- compute (x at the front f from g(f) and the
# new values of the lower neighbours), upper (u at f + 2 from b and the old
# values of the upper neighbours), relax (g at f + 1 from u and the old
# value), x memory (stages x_old [f + 4, f + 8)), x stores (stores
# [f - 4, f)), b memory (stages b [f + 3, f + 7) and the old values of the
# halo rows), poll.  The two x roles run in the same step, one reading the
# slots of [f - 4, f), the other writing those of [f + 4, f + 8), so the
# model treats them as one.  Rings: x 16 columns, b 8, u and g 4.  Values are tracked per
# (row, column) with all 5 components together.  As above, a slot written
# by one wavefront in a step must not be touched by another in that step,
# and every read a later value depends on must see the right value.
# ---------------------------------------------------------------------------
B7_TJ, B7_KT, B7_POLL, B7_PRE = 16, 4, 1, 20


def simulate_b7_tiles(shape, zero_start=False):
    nz, ny, nx = shape
    KT = B7_KT
    njt = -(-ny // B7_TJ)
    nbands = -(-nz // KT)
    # tickets in the order of the tiles' first steps j0 + k0, ties by k
    order = sorted(((jt, vt) for vt in range(nbands) for jt in range(njt)),
                   key=lambda t: (B7_TJ * t[0] + KT * t[1], t[1]))
    ticket = {t: n for n, t in enumerate(order)}
    stored = {}

    def valid(j, k):
        return 0 <= j < ny and 0 <= k < nz

    def live(j, k, c):
        return valid(j, k) and 0 <= c < nx

    def old(j, k, c):
        return ("old", j, k, c) if live(j, k, c) and not zero_start else 0

    def new(j, k, c):
        return ("new", j, k, c) if live(j, k, c) else 0

    def bval(j, k, c):
        return ("b", j, k, c) if live(j, k, c) else 0

    for vt in range(nbands):
        for jt in range(njt):
            j0, k0 = B7_TJ * jt, KT * vt
            T0 = j0 + k0
            T_start = T0 - 1 - B7_PRE
            T_lastc = T0 + (B7_TJ - 1) + (KT - 1) + nx - 1
            nblk = (T_lastc + 5 - T_start + 15) // 16
            mem = {}
            for step in range(16 * nblk):
                T = T_start + step
                p = step % 4
                # loads are parked 8 steps (two services of the plane)
                first = T - 8 < T_start
                writes, reads = [], []
                # memory wavefronts, plane p
                for e in range(320):
                    jj, cq = e // 20, (e % 20) // 5
                    j, k = j0 + jj, k0 + p
                    f = T - (j + k)
                    cs = f - 4 + cq
                    if live(j, k, cs):
                        reads.append((("x", p, jj, cs % 16), "mx",
                                      ("new", j, k, cs)))
                        stored[(k, j, cs)] = stored.get((k, j, cs), 0) + 1
                    cx = f + 4 + cq
                    writes.append((("x", p, jj, cx % 16),
                                   0 if first else old(j, k, cx), "mx"))
                    cb = f + 3 + cq
                    writes.append((("b", p, jj, cb % 8),
                                   0 if first else bval(j, k, cb), "mb"))
                for e in range(100):
                    isa = e < 20
                    hjj = 16 if isa else 4 * p + (e - 20) // 20
                    o = e if isa else (e - 20) % 20
                    hkk = p if isa else KT
                    hj, hk = j0 + hjj, k0 + hkk
                    ch = T - (hj + hk) + 4 + o // 5
                    writes.append((("x", hkk, hjj, ch % 16),
                                   0 if first else old(hj, hk, ch), "mb"))
                # poll
                for e in range(5 * (KT + 16)):
                    h = e % (KT + 16)   # records component-major
                    left = h < KT
                    jj, kk = (-1, h) if left else (h - KT, -1)
                    prod = (jt - 1, vt) if left else (jt, vt - 1)
                    ent = h if left else (KT + jj if jj < 15 else KT - 1)
                    j, k = j0 + jj, k0 + kk
                    c = T - (j + k)
                    if not (valid(j, k) and c >= 0):
                        continue
                    if c < nx:
                        assert T - B7_POLL >= T_start
                        assert ticket[prod] < ticket[(jt, vt)]
                        jp, kp = j - B7_TJ * prod[0], k - KT * prod[1]
                        pe = (kp if jp == 15 else
                              (KT + jp if kp == KT - 1 else -1))
                        assert pe == ent, (pe, ent)
                        v = ("new", j, k, c)
                    else:
                        v = 0
                    writes.append((("x", kk, jj, c % 16), v, "pl"))
                # the three arithmetic roles, lane = row (jj, kk)
                for lane in range(64):
                    jj, kk = lane & 15, lane >> 4
                    j, k = j0 + jj, k0 + kk
                    f = T - (j + k)
                    c = f + 2                       # upper
                    if live(j, k, c):
                        reads += [
                            (("b", kk, jj, c % 8), "hu", bval(j, k, c)),
                            (("x", kk, jj, (c + 1) % 16), "hu",
                             old(j, k, c + 1)),
                            (("x", kk, jj + 1, c % 16), "hu", old(j + 1, k, c)),
                            (("x", kk + 1, jj, c % 16), "hu", old(j, k + 1, c))]
                    writes.append((("u", kk, jj, c % 4),
                                   ("u", j, k, c) if live(j, k, c) else "junk",
                                   "hu"))
                    c = f + 1                       # relax
                    if live(j, k, c):
                        reads += [
                            (("u", kk, jj, c % 4), "hg", ("u", j, k, c)),
                            (("x", kk, jj, c % 16), "hg", old(j, k, c))]
                    writes.append((("g", kk, jj, c % 4),
                                   ("g", j, k, c) if live(j, k, c) else "junk",
                                   "hg"))
                    if live(j, k, f):               # compute
                        reads += [
                            (("g", kk, jj, f % 4), "cp", ("g", j, k, f)),
                            (("x", kk, jj - 1, f % 16), "cp",
                             new(j - 1, k, f)),
                            (("x", kk - 1, jj, f % 16), "cp",
                             new(j, k - 1, f))]
                        writes.append((("x", kk, jj, f % 16),
                                       ("new", j, k, f), "cp"))
                wsl = {}
                for slot, v, w in writes:
                    prev = wsl.get(slot)
                    assert prev is None or prev[1] == w, ("write race", slot)
                    wsl[slot] = (v, w)
                for slot, w, e_ in reads:
                    if slot in wsl:
                        assert wsl[slot][1] == w, ("read/write race", slot, T)
                    got = mem.get(slot, 0)
                    assert got == e_, (T, slot, got, e_)
                for slot, (v, w) in wsl.items():
                    mem[slot] = v
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                # five lanes (components) store each point's entry
                assert stored.get((k, j, i)) == 5, ("store", (k, j, i))


@pytest.mark.parametrize("shape", [(9, 7, 6), (5, 20, 11), (13, 17, 3),
                                   (1, 1, 1), (4, 33, 5), (11, 16, 8)])
def test_b7_tile_model(shape):
    simulate_b7_tiles(shape)


def test_b7_tile_model_zero_start():
    simulate_b7_tiles((6, 9, 5), zero_start=True)


def b7_tile_count(shape):
    nz, ny, nx = shape
    return -(-ny // B7_TJ) * -(-nz // B7_KT)


@pytest.mark.parametrize("shape", [(9, 7, 6), (16, 16, 16), (13, 40, 9)])
def test_b7_plan_matches_tile_model(shape):
    import paper_2204_13304_amd as m
    p = m.plan_sweep(m.block7(shape, np.eye(5)[None].repeat(7, 0) * 10))
    assert p["slab_planes"] == B7_KT
    # compute, upper, relax, x memory, poll, b memory, x stores
    assert p["threads"] == 64 * 7
    assert p["nslabs"] == b7_tile_count(shape)


# ---------------------------------------------------------------------------
# Model of the tiled VAR7 sweep kernel: the block SSOR tiles with one value
# per row and five staged arrays (x, r, x-faces, the y- and z-face below each
# row in sweep order), the row j0 + 16 (x, y-faces) and the plane k0 + KT
# (x, z-faces) as halo, one memory wavefront per compute wavefront.  Reads
# of neighbours outside the grid must give exactly 0 (they are multiplied by
# boundary faces), and every face read must give that face.
# ---------------------------------------------------------------------------
V7_TJ, V7_W, V7_PRE = 16, 8, 16


def simulate_v7_tiles(shape, nw, zero_start=False, V7_POLL=4):
    nz, ny, nx = shape
    KT = 4 * nw
    njt = -(-ny // V7_TJ)
    nbands = -(-nz // KT)
    ticket = {(jt, vt): vt * njt + jt for vt in range(nbands)
              for jt in range(njt)}
    stored = {}

    def valid(j, k):
        return 0 <= j < ny and 0 <= k < nz

    def old(j, k, c):
        if not valid(j, k) or not 0 <= c < nx or zero_start:
            return 0
        return ("old", j, k, c)

    def new(j, k, c):
        return ("new", j, k, c) if valid(j, k) and 0 <= c < nx else 0

    def arr(name, j, k, c):
        ok = {"r": valid(j, k) and 0 <= c < nx,
              "kx": valid(j, k) and 0 <= c <= nx,
              "ky": 0 <= j <= ny and 0 <= k < nz and 0 <= c < nx,
              "kz": 0 <= j < ny and 0 <= k <= nz and 0 <= c < nx}[name]
        return (name, j, k, c) if ok else 0

    for vt in range(nbands):
        for jt in range(njt):
            j0, k0 = V7_TJ * jt, KT * vt
            T0 = j0 + k0
            T_start = T0 - 1 - V7_PRE
            T_lastc = T0 + (V7_TJ - 1) + (KT - 1) + nx - 1
            nblk = (T_lastc + 5 - T_start + 15) // 16
            mem = {}

            for step in range(16 * nblk):
                T = T_start + step
                p4 = step % 4
                writes, reads = [], []
                for m in range(nw):
                    kk = 4 * m + p4
                    wm = nw + m
                    for lane in range(64):
                        jj, cq = lane >> 2, lane & 3
                        j, k = j0 + jj, k0 + kk
                        f = T - (j + k)
                        cs = f - 4 + cq
                        if valid(j, k) and 0 <= cs < nx:
                            reads.append((("x", kk, jj, cs % V7_W), wm,
                                          ("new", j, k, cs)))
                            stored[(k, j, cs)] = stored.get((k, j, cs), 0) + 1
                        c = f + 2 + cq
                        first = T - 4 < T_start
                        writes.append((("x", kk, jj, c % V7_W),
                                       0 if first else old(j, k, c), wm))
                        for a in ("r", "kx", "ky", "kz"):
                            writes.append(((a, kk, jj, c % V7_W),
                                           0 if first else arr(a, j, k, c),
                                           wm))
                        h16 = lane < 8
                        hpl = not h16 and m == nw - 1 and lane < 40
                        if not (h16 or hpl):
                            continue
                        hx = lane < 4 if h16 else ((lane - 8) >> 4) == 0
                        hjj = 16 if h16 else 4 * p4 + (((lane - 8) >> 2) & 3)
                        hkk = kk if h16 else KT
                        hj, hk = j0 + hjj, k0 + hkk
                        hc = T - (hj + hk) + 2 + cq
                        a = "x" if hx else ("ky" if h16 else "kz")
                        if first:
                            v = 0
                        elif hx:
                            v = old(hj, hk, hc)
                        else:
                            v = arr(a, hj, hk, hc)
                        writes.append(((a, hkk, hjj, hc % V7_W), v, wm))
                wp = 2 * nw
                for h in range(KT + 16):
                    left = h < KT
                    jj, kk = (-1, h) if left else (h - KT, -1)
                    prod = (jt - 1, vt) if left else (jt, vt - 1)
                    ent = h if left else (KT + jj if jj < 15 else KT - 1)
                    j, k = j0 + jj, k0 + kk
                    c = T - (j + k)
                    if not (valid(j, k) and c >= 0):
                        continue
                    if c < nx:
                        assert T - V7_POLL >= T_start
                        assert ticket[prod] < ticket[(jt, vt)]
                        jp, kp = j - V7_TJ * prod[0], k - KT * prod[1]
                        pe = (kp if jp == 15 else
                              (KT + jp if kp == KT - 1 else -1))
                        assert pe == ent, (pe, ent)
                        v = ("new", j, k, c)
                    else:
                        v = 0
                    writes.append((("x", kk, jj, c % V7_W), v, wp))
                for w in range(nw):
                    for lane in range(64):
                        jj, kk = lane & 15, 4 * w + (lane >> 4)
                        j, k = j0 + jj, k0 + kk
                        f = T - (j + k)
                        if not (valid(j, k) and 0 <= f < nx):
                            continue
                        want = [
                            (("x", kk, jj, (f + 1) % V7_W), old(j, k, f + 1)),
                            (("x", kk, jj + 1, f % V7_W), old(j + 1, k, f)),
                            (("x", kk + 1, jj, f % V7_W), old(j, k + 1, f)),
                            (("x", kk, jj - 1, f % V7_W), new(j - 1, k, f)),
                            (("x", kk - 1, jj, f % V7_W), new(j, k - 1, f)),
                            (("r", kk, jj, f % V7_W), arr("r", j, k, f)),
                            (("kx", kk, jj, f % V7_W), arr("kx", j, k, f)),
                            (("kx", kk, jj, (f + 1) % V7_W),
                             arr("kx", j, k, f + 1)),
                            (("ky", kk, jj, f % V7_W), arr("ky", j, k, f)),
                            (("ky", kk, jj + 1, f % V7_W),
                             arr("ky", j + 1, k, f)),
                            (("kz", kk, jj, f % V7_W), arr("kz", j, k, f)),
                            (("kz", kk + 1, jj, f % V7_W),
                             arr("kz", j, k + 1, f)),
                        ]
                        for slot, e_ in want:
                            reads.append((slot, w, e_))
                        writes.append((("x", kk, jj, f % V7_W),
                                       ("new", j, k, f), w))
                wsl = {}
                for slot, v, w in writes:
                    prev = wsl.get(slot)
                    assert prev is None or prev[1] == w, ("write race", slot)
                    wsl[slot] = (v, w)
                for slot, w, e_ in reads:
                    if slot in wsl:
                        assert wsl[slot][1] == w, ("read/write race", slot, T)
                    got = mem.get(slot, 0)
                    assert got == e_, (T, slot, got, e_)
                for slot, (v, w) in wsl.items():
                    mem[slot] = v
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                assert stored.get((k, j, i)) == 1, ("store", (k, j, i))


@pytest.mark.parametrize("shape", [(9, 7, 6), (5, 20, 11), (13, 17, 3),
                                   (1, 1, 1), (4, 33, 5), (17, 16, 4)])
@pytest.mark.parametrize("nw", [1, 2, 4])
@pytest.mark.parametrize("poll", [2, 4])
def test_v7_tile_model(shape, nw, poll):
    # polls 2 steps ahead when every tile has a workgroup, else 4
    simulate_v7_tiles(shape, nw, V7_POLL=poll)


def test_v7_tile_model_zero_start():
    simulate_v7_tiles((6, 9, 5), 1, zero_start=True)


@pytest.mark.parametrize("shape", [(9, 7, 6), (16, 16, 16), (13, 40, 9)])
def test_v7_plan_matches_tile_model(shape, monkeypatch):
    import torch
    import paper_2204_13304_amd as m
    nz, ny, nx = shape
    for nw in (1, 2, 4):
        monkeypatch.setenv("M2S_V7_WAVES", str(nw))
        A = _fake_var7(m, shape)
        p = m.plan_sweep(A)
        assert p["slab_planes"] == 4 * nw
        # nw compute + nw memory wavefronts + 1 poll wavefront
        assert p["threads"] == 64 * (2 * nw + 1)
        assert p["nslabs"] == -(-ny // V7_TJ) * -(-nz // (4 * nw))


# ------------------------------------------------------------------------
# The hand-off protocol of the tiled sweeps, as a CPU model: workgroups take
# tickets in the tile list's (dependency) order; a tile waits, with a
# bounded number of polls that also watch the error word, for the records
# of the tiles its lower neighbours lie in, each record carrying the epoch
# of the launch that wrote it; records are never reset between launches.
def _simulate_launch(tiles, deps, records, epoch, n_groups, spin_limit,
                     withhold=None, max_rounds=100000):
    """Round-robin over n_groups workgroups (a generator each, one action
    per turn).  Returns (tiles completed, error latched, rounds taken)."""
    state = {"ticket": 0, "err": False}
    done = set()

    def group():
        while True:
            tk = state["ticket"]
            state["ticket"] += 1
            if tk >= len(tiles) or state["err"]:
                return
            tile = tiles[tk]
            for prod in deps[tile]:
                budget = spin_limit
                while records.get(prod) != epoch:
                    budget -= 1
                    if budget < 0 or state["err"]:
                        state["err"] = True
                        break
                    yield  # sleep, then poll again
                if state["err"]:
                    break
                yield
            if state["err"]:
                continue  # back to the ticket loop, which returns
            if tile != withhold:
                records[tile] = epoch  # publish once per launch
            done.add(tile)
            yield

    gens = [group() for _ in range(n_groups)]
    rounds = 0
    while gens:
        rounds += 1
        assert rounds < max_rounds, "the launch did not drain"
        for g in list(gens):
            try:
                next(g)
            except StopIteration:
                gens.remove(g)
    return done, state["err"], rounds


def _c27_tile_graph(shape, kt):
    tiles = c27_tile_list(shape, kt)
    have = set(tiles)
    deps = {t: [p for p in ((t[0] - 1, t[1]), (t[0], t[1] - 1),
                            (t[0] - 1, t[1] - 1)) if p in have]
            for t in tiles}
    return tiles, deps


@pytest.mark.parametrize("n_groups", [1, 3, 64])
def test_protocol_completes_without_co_residency(n_groups):
    # every producer holds an earlier ticket, so the chain of waits ends at
    # a running workgroup: any number of workgroups (even one) finishes
    tiles, deps = _c27_tile_graph((23, 40, 5), 8)
    records = {}
    done, err, _ = _simulate_launch(tiles, deps, records, 1, n_groups,
                                    spin_limit=10 ** 6)
    assert not err and done == set(tiles)


@pytest.mark.parametrize("n_groups", [1, 5, 64])
def test_protocol_withheld_record_times_out_and_drains(n_groups):
    # a record that is never published (fault injection) ends every
    # workgroup with the error latched; no tile that depends on it, directly
    # or through others, completes
    tiles, deps = _c27_tile_graph((23, 40, 5), 8)
    bad = tiles[len(tiles) // 3]
    records = {}
    done, err, _ = _simulate_launch(tiles, deps, records, 1, n_groups,
                                    spin_limit=50, withhold=bad)
    assert err
    later = {t for t in tiles if t[0] >= bad[0] and t[1] >= bad[1]}
    assert not (done & (later - {bad}))


def test_protocol_records_of_an_earlier_launch_are_not_taken():
    # records are never reset: a second launch must not accept the first
    # launch's records, which carry the old epoch
    tiles, deps = _c27_tile_graph((16, 16, 16), 4)
    records = {}
    done, err, _ = _simulate_launch(tiles, deps, records, 1, 8, 10 ** 6)
    assert not err and done == set(tiles)
    bad = tiles[len(tiles) // 2]
    done, err, _ = _simulate_launch(tiles, deps, records, 2, 8, 50,
                                    withhold=bad)
    assert err and records[bad] == 1
    later = {t for t in tiles if t[0] >= bad[0] and t[1] >= bad[1]}
    assert not (done & (later - {bad}))
