"""Path-replay adjoint on the GPU against the oracle's dual-number gradient of the same
frozen-sampling estimator, and parameter updates through the C-ABI."""
import numpy as np
import pytest

from gpss_inputs import scenes as sc
from oracle import oracle as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_00280_amd import gpss
    return gpss


def _small(target, w=48, spp=4, depth=8):
    return sc.offset_sphere_scene(target, width=w, height=w, spp=spp, max_depth=depth)


def _dloss(theta0, target):
    """d/dI of mean((I - T)^2), with I and T rendered by the oracle."""
    I = orc.OracleScene(theta0).render()["mean"]
    T = orc.OracleScene(target).render()["mean"]
    return 2.0 * (I - T) / I.size


@pytest.mark.parametrize("kernel", ["persistent", "mega"])
@pytest.mark.parametrize("perturbed", [False, True])
def test_adjoint_matches_oracle_dual_gradient(G, perturbed, kernel):
    """The scheduled replay (default) and the one-thread-per-path replay against the
    oracle's forward-mode gradient of the same frozen-sampling estimator."""
    s0 = _small(False)
    if perturbed:   # theta0 with non-zero offsets, so that every gradient term is exercised
        s0.offset_grid = np.random.default_rng(9).normal(0, 0.01, s0.offset_grid.shape).astype(np.float32)
    tgt = _small(True)
    dl = _dloss(s0, tgt)
    ids = [-1, -2, -3] + [int(i) for i in sc.grad_param_indices(s0)]
    print(f"[adjoint] {kernel} perturbed={perturbed} {s0.width}x{s0.height} spp {s0.spp} params {len(ids)}",
          flush=True)
    g_orc, _ = orc.OracleScene(s0).render_grad(dl, ids)
    g = G.GpssScene(s0, kernel=kernel)
    g_off, g_sc = g.render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    torch.cuda.synchronize()
    g_off = g_off.cpu().numpy().ravel()
    g_sc = g_sc.cpu().numpy()
    g_gpu = np.array([g_sc[0], g_sc[1], g_sc[2]] + [g_off[i] for i in ids[3:]], np.float64)
    scale = np.abs(g_orc).max()
    err = np.abs(g_gpu - g_orc)
    for name, a, b in zip(["var", "len", "alb"] + [f"n{i}" for i in ids[3:]], g_gpu, g_orc):
        print(f"   {name:>8s} gpu {a:+.6e} oracle {b:+.6e}", flush=True)
    print(f"   max |diff| / max |g| = {err.max() / scale:.3e}", flush=True)
    _check_groups(g_gpu, g_orc)


@pytest.mark.parametrize("kernel", ["persistent", "mega"])
def test_adjoint_coarse_grid_contention(G, kernel):
    """A 3^3 offset grid: every gradient term of every lane lands on the same 27 nodes, so the
    workgroup table's entries are contended (its bounded swaps fall back to direct atomics)
    and evicted all the time; the gradient still equals the oracle's, all nodes compared."""
    s0 = sc.offset_sphere_scene(False, width=48, height=48, spp=8, max_depth=8, grid_res=3)
    s0.offset_grid = np.random.default_rng(11).normal(0, 0.01, s0.offset_grid.shape).astype(np.float32)
    tgt = sc.offset_sphere_scene(True, width=48, height=48, spp=8, max_depth=8, grid_res=3)
    dl = _dloss(s0, tgt)
    ids = [-1, -2, -3] + list(range(27))
    print(f"[adjoint] coarse grid {kernel} 48x48 spp 8, params {len(ids)}", flush=True)
    g_orc, _ = orc.OracleScene(s0).render_grad(dl, ids)
    g = G.GpssScene(s0, kernel=kernel)
    g_off, g_sc = g.render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    torch.cuda.synchronize()
    g_off = g_off.cpu().numpy().ravel()
    g_sc = g_sc.cpu().numpy()
    g_gpu = np.array([g_sc[0], g_sc[1], g_sc[2]] + [g_off[i] for i in ids[3:]], np.float64)
    _check_groups(g_gpu, g_orc)


def _check_groups(g_gpu, g_ref, rel=1e-4, floor=1e-6):
    """Per parameter, scalars and grid nodes as separate groups: |gpu - ref| at most rel x |ref|,
    or at most floor x the group's largest |ref| for entries near zero."""
    assert np.isfinite(g_gpu).all()
    for sl in (slice(0, 3), slice(3, None)):
        a, b = np.asarray(g_gpu[sl], np.float64), np.asarray(g_ref[sl], np.float64)
        scale = np.abs(b).max()
        assert scale > 0
        tol = np.maximum(rel * np.abs(b), floor * scale)
        err = np.abs(a - b)
        worst = int(np.argmax(err / tol))
        assert (err <= tol).all(), (sl, worst, a[worst], b[worst], float(err[worst] / tol[worst]))


def test_adjoint_full_size_sampled_pixels(G):
    """The offset-sphere workload at full size (256^2, 16 spp, depth 16): loss weight on 400
    random pixels, so the oracle traces only those; all 32 parameters compared."""
    s0 = sc.offset_sphere_scene(False)
    rng = np.random.default_rng(21)
    dl = np.zeros((s0.height, s0.width))
    ys, xs = np.meshgrid(np.arange(64, 192), np.arange(64, 192), indexing="ij")
    pick = rng.choice(ys.size, 400, replace=False)
    dl[ys.ravel()[pick], xs.ravel()[pick]] = rng.normal(size=400) / s0.n_pixels
    ids = [-1, -2, -3] + [int(i) for i in sc.grad_param_indices(s0)]
    print(f"[adjoint] full size {s0.width}x{s0.height} spp {s0.spp} depth {s0.max_depth}", flush=True)
    g_orc, _ = orc.OracleScene(s0).render_grad(dl, ids, want_image=False)
    g_off, g_sc = G.GpssScene(s0).render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    g_off = g_off.cpu().numpy().ravel()
    g_sc = g_sc.cpu().numpy()
    g_gpu = np.array(list(g_sc) + [g_off[i] for i in ids[3:]], np.float64)
    print("   scalars gpu", g_gpu[:3], "oracle", g_orc[:3], flush=True)
    print("   nodes: nonzero", int((g_orc[3:] != 0).sum()), "max rel",
          float(np.max(np.abs(g_gpu[3:] - g_orc[3:])) / np.abs(g_orc[3:]).max()), flush=True)
    _check_groups(g_gpu, g_orc)


def test_set_params_equals_fresh_scene(G):
    s0 = _small(False, w=32)
    tgt = _small(True, w=32)
    g = G.GpssScene(s0)
    off = torch.as_tensor(tgt.offset_grid, device="cuda")
    g.set_params(off, tgt.variance, tgt.lengthscale, tgt.albedo)
    a = g.render().cpu().numpy()
    fresh = G.GpssScene(tgt)
    b = fresh.render().cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(g.majorants(), fresh.majorants())


def test_adjoint_without_offset_grid(G):
    s = sc.sphere_scene(0.1, width=32, height=32, spp=4, max_depth=8)
    dl = np.random.default_rng(1).normal(size=(32, 32)) / 1024
    ids = [-1, -2, -3]
    g_orc, _ = orc.OracleScene(s).render_grad(dl, ids)
    g_off, g_sc = G.GpssScene(s).render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    assert g_off is None
    g_sc = g_sc.cpu().numpy().astype(np.float64)
    print("   gpu", g_sc, "oracle", g_orc, flush=True)
    assert np.isfinite(g_sc).all()
    tol = np.maximum(1e-4 * np.abs(g_orc), 1e-6 * np.abs(g_orc).max())
    assert (np.abs(g_sc - g_orc) <= tol).all(), (g_sc, g_orc)


def test_torch_autograd_function(G):
    from paper_2603_00280_amd import autograd as ag
    s0 = _small(False, w=32)
    tgt = _small(True, w=32)
    T = G.GpssScene(tgt).render()
    scene = G.GpssScene(s0)
    off = torch.zeros(s0.offset_grid.shape, device="cuda", requires_grad=True)
    var = torch.tensor(float(np.float32(s0.variance)), requires_grad=True)
    ls = torch.tensor(float(np.float32(s0.lengthscale)), requires_grad=True)
    alb = torch.tensor(float(np.float32(s0.albedo)), requires_grad=True)
    img = ag.render(scene, off, var, ls, alb)
    loss = ((img - T) ** 2).mean()
    loss.backward()
    dl = (2.0 * (img.detach() - T) / img.numel())
    g_off, g_sc = scene.render_adjoint(dl)
    assert var.grad.device.type == "cpu" and off.grad.device.type == "cuda"
    assert torch.allclose(off.grad, g_off, rtol=1e-5, atol=1e-9)
    got = torch.stack([var.grad, ls.grad, alb.grad]).float()
    assert torch.allclose(got, g_sc.cpu(), rtol=1e-5, atol=1e-9)


def test_gradient_descent_reduces_loss(G):
    """A few Adam steps on (variance, lengthscale, albedo) toward the target's values."""
    from paper_2603_00280_amd import autograd as ag
    s0 = sc.sphere_scene(0.12, width=48, height=48, spp=8, max_depth=8, variance=0.003, albedo=0.7)
    tgt = sc.sphere_scene(0.1, width=48, height=48, spp=8, max_depth=8, variance=0.0025, albedo=0.8)
    T = G.GpssScene(tgt).render()
    scene = G.GpssScene(s0)
    # optimise the logarithms of the three parameters (they differ by orders of magnitude)
    p = torch.log(torch.tensor([0.003, 0.12, 0.7], dtype=torch.float64)).requires_grad_(True)
    opt = torch.optim.Adam([p], lr=0.03)
    losses = []
    for _ in range(8):
        opt.zero_grad()
        q = torch.exp(p)
        img = ag.render(scene, None, q[0], q[1], q[2].clamp(max=1.0))
        loss = ((img - T) ** 2).mean()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    print("   losses", [f"{l:.3e}" for l in losses], flush=True)
    assert losses[-1] < losses[0]


def test_adjoint_matches_central_differences(G):
    """The default adjoint on 32 parameters (variance, lengthscale, albedo and 29 offset-grid
    nodes near the surface) against FP64 central differences (h = 1e-4 relative for the
    scalars, 1e-5 for the nodes) of the oracle's frozen-sampling estimator at theta0."""
    from tests.test_oracle_pins import _unrounded
    s0 = _small(False)
    s0.offset_grid = np.random.default_rng(9).normal(0, 0.01, s0.offset_grid.shape).astype(np.float32)
    dl = _dloss(s0, _small(True))
    ids = [-1, -2, -3] + [int(i) for i in sc.grad_param_indices(s0)]
    assert len(ids) == 32
    base = orc.OracleScene(s0)
    h = 1e-4
    fd = []
    for pid in ids:
        imgs = []
        for sgn in (+1, -1):
            if pid in (-1, -2, -3):
                field = {-1: "variance", -2: "lengthscale", -3: "albedo"}[pid]
                v = float(orc.f32(getattr(s0, field)))
                pert = s0.replace(**{field: v * (1 + sgn * h)})
                scale = v * h
            else:
                off = s0.offset_grid.astype(np.float64).copy()
                off.ravel()[pid] += sgn * 1e-5
                pert = s0.replace(offset_grid=off.astype(np.float32))
                scale = abs(float(np.float32(off.ravel()[pid])) - float(s0.offset_grid.ravel()[pid]))
            imgs.append(base.render_frozen(_unrounded(pert)))
        fd.append(float(np.sum(dl * (imgs[0] - imgs[1]))) / (2 * scale))
    fd = np.array(fd)
    print(f"[adjoint] central differences, {len(ids)} parameters", flush=True)
    g = G.GpssScene(s0)
    g_off, g_sc = g.render_adjoint(torch.as_tensor(dl, dtype=torch.float32))
    torch.cuda.synchronize()
    g_off = g_off.cpu().numpy().ravel()
    g_sc = g_sc.cpu().numpy()
    g_gpu = np.array([g_sc[0], g_sc[1], g_sc[2]] + [g_off[i] for i in ids[3:]], np.float64)
    for name, a, b in zip(["var", "len", "alb"] + [f"n{i}" for i in ids[3:]], g_gpu, fd):
        print(f"   {name:>8s} gpu {a:+.6e} fd {b:+.6e}", flush=True)
    _check_groups(g_gpu, fd)


def test_adjoint_full_size_central_differences(G):
    """The offset-sphere workload at its full size (256^2, 16 spp, depth 16) with the L2 loss
    restricted to 4000 pixels sampled over the sphere's image: the GPU adjoint on its 32
    parameters against the oracle's dual-number gradient and against FP64 central differences
    (h = 1e-4 relative for the scalars, 1e-5 for the nodes) of the oracle's frozen-sampling
    estimator on those pixels; the oracle's two gradients against each other as well."""
    from tests.test_oracle_pins import _unrounded
    s0 = sc.offset_sphere_scene(False)
    tgt = sc.offset_sphere_scene(True)
    rng = np.random.default_rng(31)
    ys, xs = np.meshgrid(np.arange(48, 208), np.arange(48, 208), indexing="ij")
    px = np.sort((ys.ravel() * s0.width + xs.ravel())[rng.choice(ys.size, 4000, replace=False)])
    I = orc.OracleScene(s0).render_pixels(px)["mean"]
    T = orc.OracleScene(tgt).render_pixels(px)["mean"]
    dl = np.zeros(s0.n_pixels)
    dl[px] = 2.0 * (I - T) / px.size
    ids = [-1, -2, -3] + [int(i) for i in sc.grad_param_indices(s0)]
    assert len(ids) == 32
    print(f"[adjoint] full-size central differences, {px.size} pixels, {len(ids)} parameters", flush=True)
    g_orc, _ = orc.OracleScene(s0).render_grad(dl, ids, want_image=False)
    base = orc.OracleScene(s0)
    fd = []
    for pid in ids:
        vals = []
        for sgn in (+1, -1):
            if pid < 0:
                field = {-1: "variance", -2: "lengthscale", -3: "albedo"}[pid]
                v = float(orc.f32(getattr(s0, field)))
                pert = s0.replace(**{field: v * (1 + sgn * 1e-4)})
                scale = v * 1e-4
            else:
                off = s0.offset_grid.astype(np.float64).copy()
                off.ravel()[pid] += sgn * 1e-5
                pert = s0.replace(offset_grid=off.astype(np.float32))
                scale = abs(float(np.float32(off.ravel()[pid])) - float(s0.offset_grid.ravel()[pid]))
            vals.append(base.render_frozen_pixels(_unrounded(pert), px))
        fd.append(float(np.sum(dl[px] * (vals[0] - vals[1]))) / (2 * scale))
    fd = np.array(fd)
    g_off, g_sc = G.GpssScene(s0).render_adjoint(torch.as_tensor(dl.reshape(s0.height, s0.width),
                                                                 dtype=torch.float32))
    torch.cuda.synchronize()
    g_off = g_off.cpu().numpy().ravel()
    g_gpu = np.array(list(g_sc.cpu().numpy()) + [g_off[i] for i in ids[3:]], np.float64)
    for name, a, b, c in zip(["var", "len", "alb"] + [f"n{i}" for i in ids[3:]], g_gpu, g_orc, fd):
        print(f"   {name:>8s} gpu {a:+.6e} oracle {b:+.6e} fd {c:+.6e}", flush=True)
    assert np.count_nonzero(fd[3:]) >= 20      # the sampled pixels reach most of the nodes
    _check_groups(g_orc, fd, rel=1e-5, floor=1e-8)
    _check_groups(g_gpu, g_orc)
    _check_groups(g_gpu, fd)


def test_adjoint_keeps_nothing_per_path(G):
    """The adjoint replays each path in the lane that traced it: a call over 64 times the paths
    of a first call (1024^2 x 64 spp, 67 M paths) takes no device memory beyond the first
    call's, where one float per path would be 256 MiB."""
    s = sc.offset_sphere_scene(False, width=1024, height=1024, spp=64)
    g = G.GpssScene(s)
    dl = torch.full((s.height, s.width), 1e-6, dtype=torch.float32, device="cuda")
    g.render_adjoint(dl, 0, 1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    print(f"[adjoint memory] {s.n_paths} paths", flush=True)
    g_off, g_sc = g.render_adjoint(dl, 0, 64)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (32 << 20)
    assert torch.isfinite(g_off).all() and torch.isfinite(g_sc).all()
