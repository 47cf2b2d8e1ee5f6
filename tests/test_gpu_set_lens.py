"""raysh_set_lens: a context given another lens maps exactly as a new
context of that lens, in every precision, through growth and shrinking of
its star buffer, with star cells and captured batches rebuilt, and keeps
its lens when the new one is rejected."""
import numpy as np
import pytest

from paper_1703_09707_amd import raysh as R
from paper_1703_09707_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    return t


def _lens(n, seed, kappa_c=0.1, g1=0.25, g2=-0.05):
    rng = np.random.default_rng(seed)
    m = W.salpeter_masses(n, rng) if n else np.zeros(0)
    x = rng.uniform(-12, 12, n)
    y = rng.uniform(-12, 12, n)
    return (kappa_c, g1, g2, x, y, m)


def _rays():
    return W.centred_rays(14.0, 14.0, 640, 512)


def _pix():
    return W.centred_window(10.0, 256)


def _fresh(torch, lens, prec, cells="auto"):
    with R.Context(lens) as ctx:
        ctx.set_expansion_cells(cells)
        return ctx.map(_rays(), _pix(), prec).cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32_bulk", "fp64_expansion"])
def test_set_lens_maps_as_a_new_context(torch, prec):
    print("set_lens", prec, flush=True)
    lenses = [_lens(300, 1), _lens(2000, 2, 0.2), _lens(50, 3, 0.0, 0.4, 0.1), _lens(0, 4), _lens(3000, 5)]
    with R.Context(lenses[0]) as ctx:
        first = ctx.map(_rays(), _pix(), prec).cpu().numpy()
        np.testing.assert_array_equal(first, _fresh(torch, lenses[0], prec))
        for lens in lenses[1:]:   # grows (300 -> 2000), shrinks, no stars, grows again
            ctx.set_lens(lens)
            got = ctx.map(_rays(), _pix(), prec).cpu().numpy()
            np.testing.assert_array_equal(got, _fresh(torch, lens, prec))
            assert ctx.n_stars == len(lens[3])


def test_set_lens_rebuilds_star_cells(torch):
    a, b = _lens(800, 11), _lens(1200, 12, 0.2)
    with R.Context(a) as ctx:
        ctx.set_expansion_cells("always")
        ctx.map(_rays(), _pix(), "fp64_expansion")     # builds a's cells
        ctx.set_lens(b)
        got = ctx.map(_rays(), _pix(), "fp64_expansion").cpu().numpy()
    np.testing.assert_array_equal(got, _fresh(torch, b, "fp64_expansion", cells="always"))


def test_set_lens_drops_captured_batches(torch):
    lenses = [_lens(400, 21), _lens(900, 22, 0.3)]
    new = _lens(1500, 23, -0.1)
    ctxs = [R.Context(l) for l in lenses]
    try:
        rays, pix = [_rays()] * 2, [_pix()] * 2
        before = [m.cpu().numpy() for m in R.map_batch(ctxs, rays, pix, "fp64")]
        for m, l in zip(before, lenses):
            np.testing.assert_array_equal(m, _fresh(torch, l, "fp64"))
        R.map_batch(ctxs, rays, pix, "fp64")          # replayed from the captured graph
        ctxs[1].set_lens(new)
        after = [m.cpu().numpy() for m in R.map_batch(ctxs, rays, pix, "fp64")]
        np.testing.assert_array_equal(after[0], before[0])
        np.testing.assert_array_equal(after[1], _fresh(torch, new, "fp64"))
    finally:
        for c in ctxs:
            c.close()


def test_set_lens_rejected_keeps_the_old_lens(torch):
    a = _lens(500, 31)
    bad = list(_lens(500, 32))
    bad[3] = bad[3].copy()
    bad[3][7] = np.nan
    with R.Context(a) as ctx:
        with pytest.raises(R.RayshError):
            ctx.set_lens(tuple(bad))
        got = ctx.map(_rays(), _pix(), "fp64").cpu().numpy()
    np.testing.assert_array_equal(got, _fresh(torch, a, "fp64"))
