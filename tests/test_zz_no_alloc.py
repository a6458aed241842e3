"""gpss_render_noalloc through the C-ABI: its scratch lives in the library's fixed device array,
and its images equal gpss_render's bit for bit (same paths, same fixed-point sums).  Two calls
in a row, the second on a smaller image, so that what the first left in the shared array
beyond the second image's pixels cannot leak into it; the size limit is rejected."""
import ctypes as C

import numpy as np
import pytest

from gpss_inputs import scenes as sc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_00280_amd import gpss
    return gpss


def _noalloc(G, g, s0=0, s1=None):
    s1 = g.scene.spp if s1 is None else s1
    out = torch.full(g.shape, -1.0, dtype=torch.float32, device="cuda")
    G.gpss_render_noalloc(g.handle, out.data_ptr(), s0, s1)
    return out


def test_noalloc_matches_render_twice_second_smaller(G):
    big = G.GpssScene(sc.sphere_scene(0.02, width=96, height=80, spp=8, max_depth=16))
    small = G.GpssScene(sc.mixed_scene(width=40, height=24, spp=4, max_depth=16))
    for g in (big, small):
        print(f"[noalloc] {g.scene.name} {g.scene.width}x{g.scene.height} spp {g.scene.spp}", flush=True)
        a = _noalloc(G, g)
        b = g.render()
        torch.cuda.synchronize()
        assert torch.equal(a, b), (g.scene.name, float((a - b).abs().max()))
        assert float(a.abs().sum()) > 0.0


def test_noalloc_sample_range_and_repeat(G):
    g = G.GpssScene(sc.sphere_scene(0.1, width=64, height=48, spp=12, max_depth=8))
    r1 = _noalloc(G, g, 3, 9)
    r2 = _noalloc(G, g, 3, 9)
    ref = g.render(3, 9)
    torch.cuda.synchronize()
    assert torch.equal(r1, ref) and torch.equal(r2, ref)


def test_noalloc_rejects_images_beyond_its_array(G):
    s = sc.sphere_scene(0.1, width=1025, height=1024, spp=1, max_depth=2)
    g = G.GpssScene(s)
    out = torch.empty(g.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GpssError) as e:
        G.gpss_render_noalloc(g.handle, out.data_ptr(), 0, 1)
    assert e.value.code == -1 and "at most 1048576" in str(e.value)
    # the largest image it holds renders
    g2 = G.GpssScene(sc.sphere_scene(0.1, width=1024, height=1024, spp=1, max_depth=2))
    a = _noalloc(G, g2)
    b = g2.render()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
