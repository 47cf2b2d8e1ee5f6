"""The FMA probe (a measurement aid): its values are exact, so a launch that
ran every FMA it claims is checked element by element."""
import pytest

from paper_1703_09707_amd import raysh as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return t


@pytest.mark.parametrize("prec", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("blocks,iters", [(1, 1), (3, 7), (512, 1000)])
def test_fma_probe_values(torch, prec, blocks, iters):
    print("fma probe", prec, blocks, iters, flush=True)
    out = R.fma_probe(prec, blocks, iters)
    torch.cuda.synchronize()
    lane = torch.arange(blocks * 256, device="cuda") % 64
    want = (8 * (lane + iters) + 28).to(out.dtype)   # sum over chains i < 8 of (lane + i + iters)
    assert torch.equal(out, want)


def test_fma_probe_rejects_a_short_buffer(torch):
    # the check is against the buffer's allocation (a caching allocator's
    # segment may be larger than the tensor): ask for far more than any
    buf = torch.zeros(100, dtype=torch.float64, device="cuda")
    import ctypes
    lib = R.load()
    code = lib.raysh_fma_probe(R.FP64, 1 << 22, 4, ctypes.c_void_p(buf.data_ptr()), None)   # 8 GiB
    assert code == R.EINVAL and "out" in lib.raysh_last_error().decode()
    assert bool((buf == 0).all())
