"""GPU parity of the line-scheduled 27-point sweep with the x-line affine
scan (m2s_symgs_xline) against the oracle's exact lexicographic sweep.
The scan regroups the sums along each line, so the bar is relative 1e-13
in FP64, not bitwise."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13304_amd import inputs
from tests.gpu_util import banner, dev, host, rel_inf

pytestmark = pytest.mark.gpu

# (nz, ny, nx): single points and lines, ragged shapes, lines longer than
# the 256-thread workgroup (several points per scan chunk, ragged chunks)
SHAPES = [(16, 16, 16), (9, 26, 13), (1, 1, 1), (1, 1, 300), (2, 3, 70),
          (70, 3, 2), (5, 1, 8), (3, 4, 600), (12, 5, 257), (24, 24, 24)]


@pytest.fixture(scope="module")
def m():
    import paper_2204_13304_amd as pkg
    assert torch.cuda.is_available()
    return pkg


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_xline_parity(m, shape, direction):
    banner(f"symgs27 x-line scan {direction} {shape}")
    A = m.const27(shape)
    ws = m.Workspace(A)
    r = inputs.standard_normal(60, shape)
    x0 = inputs.standard_normal(61, shape)
    xg = dev(x0)
    m.symgs_xline(A, dev(r), xg, direction, ws)
    ws.check()
    assert rel_inf(host(xg), oracle.symgs27(r, x0, direction)) <= 1e-13


def test_xline_shares_workspace_with_wavefront(m):
    # the line sweep and the tiled sweep take tickets from one counter
    shape = (21, 19, 23)
    banner("symgs27 x-line / wavefront alternation")
    A = m.const27(shape)
    ws = m.Workspace(A)
    r = inputs.standard_normal(62, shape)
    x0 = inputs.standard_normal(63, shape)
    xg = dev(x0)
    ref = x0
    for step in range(3):
        m.symgs_xline(A, dev(r), xg, "sym", ws)
        m.symgs(A, dev(r), xg, "sym", ws)
        ref = oracle.symgs27(r, oracle.symgs27(r, ref, "sym"), "sym")
    ws.check()
    assert rel_inf(host(xg), ref) <= 1e-13


@pytest.mark.parametrize("n", [104, 256])
def test_xline_full_size(m, n):
    shape = (n, n, n)
    banner(f"symgs27 x-line full size {shape}")
    A = m.const27(shape)
    ws = m.Workspace(A)
    r = inputs.standard_normal(10, shape)
    x0 = inputs.standard_normal(11, shape)
    xg = dev(x0)
    m.symgs_xline(A, dev(r), xg, "sym", ws)
    ws.check()
    assert rel_inf(host(xg), oracle.symgs27(r, x0, "sym")) <= 1e-13


def test_xline_rejects_other_kinds_and_f32(m):
    A32 = m.const27((8, 8, 8), dtype=torch.float32)
    x = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        m.symgs_xline(A32, x.clone(), x)
    A = m.const27((4, 4, 5000))
    x = torch.zeros((4, 4, 5000), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        m.symgs_xline(A, x.clone(), x)


def test_xline_wait_timeout_is_reported_and_recovered(m, monkeypatch):
    # a spin limit of one poll makes a plane give up waiting for the plane
    # below: every workgroup exits, the latch reports the time-out, and the
    # workspace is usable afterwards
    shape = (12, 40, 9)
    banner("symgs27 x-line forced wait time-out")
    A = m.const27(shape)
    ws = m.Workspace(A)
    r = inputs.standard_normal(64, shape)
    x0 = inputs.standard_normal(65, shape)
    monkeypatch.setenv("M2S_SPIN_LIMIT", "1")
    m.symgs_xline(A, dev(r), dev(x0), "fwd", ws)
    with pytest.raises(RuntimeError, match="M2S_ERR_TIMEOUT"):
        ws.check()
    monkeypatch.delenv("M2S_SPIN_LIMIT")
    xg = dev(x0)
    m.symgs_xline(A, dev(r), xg, "sym", ws)
    ws.check()
    assert rel_inf(host(xg), oracle.symgs27(r, x0, "sym")) <= 1e-13
    xg = dev(x0)
    m.symgs(A, dev(r), xg, "sym", ws)
    assert rel_inf(host(xg), oracle.symgs27(r, x0, "sym")) <= 1e-13
