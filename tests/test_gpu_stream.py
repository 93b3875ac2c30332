"""GPU check of the STREAM reference kernels (measurement support, not a
step of the method): copy and triad against torch on even and odd lengths,
and the argument checks."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 7, 4096, 1_000_001])
def test_stream_copy_and_triad(n):
    import paper_2204_13304_amd as m
    a = torch.randn(n, dtype=torch.float64, device="cuda")
    b = torch.randn(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    m.stream("copy", a, c)
    assert torch.equal(c, a)
    m.stream("triad", a, c, b, 3.0)
    assert torch.equal(c, a + 3.0 * b)


def test_stream_rejects_overlap_and_misalignment():
    import paper_2204_13304_amd as m
    a = torch.randn(64, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="M2S_ERR_ALIAS"):
        m.stream("copy", a[:32], a[16:48])
    with pytest.raises(RuntimeError, match="M2S_ERR_ARG"):
        m.stream("copy", a[1:33], a[32:64])
