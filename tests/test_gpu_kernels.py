"""The wavefront and the persistent scheduled tracers against the one-thread-per-path
kernel: identical arithmetic per path, so path radiances must agree bit for bit, and event
counts must be equal."""
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


CASES = {
    "plane": lambda: sc.plane_scene(),
    "sphere_l0.005": lambda: sc.sphere_scene(0.005, width=64, height=64, spp=4),
    "sphere_l0.5": lambda: sc.sphere_scene(0.5, width=64, height=64, spp=4),
    "mixed": lambda: sc.mixed_scene(width=48, height=48, spp=2),
    "offset": lambda: sc.offset_sphere_scene(True, width=48, height=48, spp=4),
    "ragged": lambda: sc.sphere_scene(0.02, width=37, height=23, spp=3, max_depth=5),
    "furnace": lambda: sc.plane_scene(width=16, height=16, spp=8, max_depth=40, albedo=1.0,
                                      env=1.0, light_E=0.0),
    "aniso_sphere": lambda: sc.aniso_sphere_scene(0.01, width=48, height=48, spp=4),
    "ggx_sphere": lambda: sc.ggx_sphere_scene(0.3, width=48, height=48, spp=4),
}


@pytest.mark.parametrize("kernel", ["wavefront", "persistent"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_kernel_matches_megakernel_bitwise(G, name, kernel):
    s = CASES[name]()
    print(f"[{kernel}] {name} {s.width}x{s.height} spp {s.spp} depth {s.max_depth}", flush=True)
    g = G.GpssScene(s, kernel="mega")
    pm, cm = g.render_paths(counters=True)
    g.set_kernel(kernel)
    pw, cw = g.render_paths(counters=True)
    pm, pw = pm.cpu().numpy(), pw.cpu().numpy()
    diff = np.flatnonzero(pm.view(np.uint32) != pw.view(np.uint32))
    assert diff.size == 0, (diff[:8], pm.ravel()[diff[:8]], pw.ravel()[diff[:8]])
    assert G.counters_dict(cm) == G.counters_dict(cw)
    # every path radiance is a finite, non-negative estimate below the accumulator's range
    assert G.counters_dict(cm)["nonfinite"] == 0 and G.counters_dict(cm)["saturated"] == 0
    # the image entry point through both kernels
    im_w = g.render().cpu().numpy()
    g.set_kernel("mega")
    im_m = g.render().cpu().numpy()
    assert np.array_equal(im_w, im_m)


@pytest.mark.parametrize("kernel", ["wavefront", "persistent"])
def test_sample_ranges_and_reuse(G, kernel):
    s = sc.sphere_scene(0.1, width=40, height=24, spp=12, max_depth=8)
    g = G.GpssScene(s, kernel=kernel)
    full = g.render_paths(0, 12).cpu().numpy()
    a = g.render_paths(0, 5).cpu().numpy()
    b = g.render_paths(5, 12).cpu().numpy()
    assert np.array_equal(np.concatenate([a, b], axis=2), full)
    # a larger launch after a smaller one, then a smaller one again (buffer reuse)
    big = G.GpssScene(s.replace(width=64, height=64), kernel=kernel)
    big.render_paths(0, 12)
    again = g.render_paths(0, 12).cpu().numpy()
    assert np.array_equal(again, full)


def test_auto_is_persistent_and_single_path_launches(G):
    """The default kernel is the persistent one; launches smaller than one wave's chunk
    (a single path, a 1x1 image) and larger than the resident grid both complete."""
    s = sc.sphere_scene(0.02, width=1, height=1, spp=1, max_depth=6)
    g = G.GpssScene(s)
    p1 = g.render_paths().cpu().numpy()
    g.set_kernel("mega")
    assert np.array_equal(p1, g.render_paths().cpu().numpy())
