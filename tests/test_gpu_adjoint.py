"""GPU path-replay VJP vs the oracle's FP64 reverse sweep, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes
from .gpu_util import GRAD_KEYS, VJP_MODES, GpuRun, compare_grads, ctx, dev, run_vjp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    O.build(force=False)


def _clean_cotangent(w, seed, sc):
    """Random cotangent, zero on pixels with a sample near a decision boundary
    (hit, frustum, sign or clip threshold): there FP32 and FP64 may legitimately differ."""
    ref = O.render(sc, want=("margin_clip",))
    allc = (ref["margin_clip"] >= 1).all(axis=1)
    assert allc.mean() > 0.9
    G = np.random.default_rng(seed).normal(size=(w.camera.height * w.camera.width, 3))
    G[~allc] = 0.0
    return G.reshape(w.camera.height, w.camera.width, 3)


@pytest.mark.parametrize("clip,env", [(False, False), (True, False), (True, True)])
def test_vjp_matches_oracle_ggx(clip, env):
    w = scenes.c3_ggx(spp=4, seed=21, max_depth=3)
    w.clip = clip
    w.clip_k = 0.5
    if env:
        w.env = np.array([0.04, 0.06, 0.05])
    sc = O.Scene(w)
    G = _clean_cotangent(w, 5, sc)
    ref = O.render_vjp(sc, G)
    run = GpuRun(w)
    for mode in VJP_MODES:   # own records, caller's records, re-tracing replay
        gpu = run_vjp(run, G, mode=mode)
        worst = compare_grads(gpu, ref)
        print(f"{mode}: worst global relative gradient error {worst:.2e}")


@pytest.mark.parametrize("depth", [1, 9])
def test_vjp_direct_only_and_deep_paths(depth):
    """Depth 1 (direct light only: no bounce, no pending cotangents) and depth 9, whose
    replay flushes its binned map cotangents three times (after depths 4, 8 and 9) and
    carries pending cotangents across each flush, with the environment light on."""
    w = scenes.c3_ggx(spp=4, seed=41, max_depth=depth)
    w.env = np.array([0.05, 0.04, 0.06])
    sc = O.Scene(w)
    G = _clean_cotangent(w, 7, sc)
    ref = O.render_vjp(sc, G)
    run = GpuRun(w)
    for mode in VJP_MODES:
        worst = compare_grads(run_vjp(run, G, mode=mode), ref)
        print(f"depth {depth} {mode}: worst global relative gradient error {worst:.2e}")


def test_vjp_deep_paths_in_a_corner():
    """Depth 8 in the folded corner (concave: paths keep bouncing between floor and wall,
    so every depth holds records and two full flushes run), 512^2 GGX maps, env on."""
    from paper_2503_12174_amd import dpcs
    w = synth.corner_50k(spp=8, max_depth=8, res=48, n_quads=10, env=0.05)
    sc = O.Scene(w)
    hits = O.render(sc, want=("hits",))["hits"]
    assert (hits[:, :, 5] >= 0).sum() >= 10   # records past the first flush
    G = _clean_cotangent(w, 9, sc)
    ref = O.render_vjp(sc, G)
    run = GpuRun(w, scene=dpcs.Scene(ctx(), w.mesh, bvh="sah"))
    for mode in VJP_MODES:
        worst = compare_grads(run_vjp(run, G, mode=mode), ref)
        print(f"corner depth 8 {mode}: worst global relative gradient error {worst:.2e}")


def test_vjp_non_square_devices_and_maps():
    """Camera, projector and maps of different, non-square sizes (the capture aspect
    ratios of the paper's setup, scaled down): a swapped width and height anywhere in
    the projector image, the maps or their gradients fails here."""
    import math
    w = scenes.c3_ggx(spp=4, seed=31, max_depth=3)
    w.camera = synth.pinhole((0, 0, 0.8), (0, 0, 0), 60.0, 64, 36, up=(0, 1, 0))
    ang = math.radians(30.0)
    w.projector = synth.pinhole((-0.6 * math.sin(ang), 0.0, 0.6 * math.cos(ang)), (0, 0, 0), 60.0, 80, 60,
                                up=(0, 1, 0))
    rng = np.random.default_rng(32)
    w.proj_image = rng.uniform(0, 1, (60, 80, 3)).astype(np.float32)
    w.albedo = rng.uniform(0.2, 0.8, (24, 40, 3)).astype(np.float32)
    w.roughness = rng.uniform(0.2, 0.9, (24, 40)).astype(np.float32)
    w.specular = rng.uniform(0.0, 1.0, (24, 40)).astype(np.float32)
    w.env = np.array([0.03, 0.04, 0.05])
    sc = O.Scene(w)
    G = _clean_cotangent(w, 33, sc)
    ref = O.render_vjp(sc, G)
    run = GpuRun(w)
    for mode in VJP_MODES:
        compare_grads(run_vjp(run, G, mode=mode), ref)


@pytest.mark.parametrize("mode", VJP_MODES)
def test_vjp_is_deterministic(mode):
    """Three VJP calls on the same inputs give bit-identical gradients: the map
    cotangents are summed exactly in fixed point (chunk sums kept as integers, so the
    order in which atomics placed the records does not matter) and the scalar partials
    are reduced in a fixed order.  The 50k-triangle corner at 96^2 x 16 spp spreads each
    tile's records over several accumulation chunks."""
    w = synth.corner_50k(spp=16, res=96)
    G = np.random.default_rng(41).normal(size=(96, 96, 3))
    run = GpuRun(w)
    outs = [run_vjp(run, G, mode=mode) for _ in range(3)]
    for k in GRAD_KEYS:
        for o in outs[1:]:
            assert np.array_equal(np.asarray(o[k]), np.asarray(outs[0][k])), k
    assert np.abs(outs[0]["albedo"]).max() > 0 and np.abs(outs[0]["Ip"]).max() > 0


def test_vjp_lambert_quad_cube():
    w = synth.quad_cube()
    sc = O.Scene(w)
    G = _clean_cotangent(w, 6, sc)
    ref = O.render_vjp(sc, G)
    gpu = run_vjp(GpuRun(w), G)
    compare_grads(gpu, ref, keys=("Ip", "albedo", "prf_gamma", "prf_mix", "crf_gamma", "white_balance"))
    assert np.abs(gpu["roughness"]).max() == 0 and np.abs(gpu["specular"]).max() == 0


def test_vjp_with_stored_samples_equals_recomputed():
    import torch
    from paper_2503_12174_amd import dpcs
    w = scenes.c3_ggx(spp=4, seed=2, max_depth=3)
    run = GpuRun(w)
    H, W = 64, 64
    L = torch.zeros((H, W, w.spp, 3), device="cuda")
    out = torch.zeros((H, W, 3), device="cuda")
    dpcs.dpcs_render(run.c, run.scene, run.params, run.proj, out, sample_radiance=L)
    G = np.random.default_rng(3).normal(size=(H, W, 3))
    a = run_vjp(run, G)
    b = run_vjp(run, G, sample_radiance=L)
    for k in a:
        np.testing.assert_allclose(a[k], b[k], rtol=1e-4, atol=1e-6 * (np.abs(a[k]).max() + 1e-30))


def test_vjp_dot_product_on_linear_map():
    """<G, R(v)> == <R^T G, v> for the linear configuration, all on the GPU."""
    w = scenes.linear_params(scenes.c3_ggx(spp=4, seed=8, max_depth=3))
    v = np.random.default_rng(1).uniform(0, 1, w.proj_image.shape).astype(np.float32)
    run = GpuRun(w, proj_image=v)
    Av = run.render()["Ic"].reshape(64, 64, 3).astype(np.float64)
    G = np.random.default_rng(2).normal(size=(64, 64, 3))
    g = run_vjp(run, G)
    lhs = (G * Av).sum()
    rhs = (g["Ip"] * v).sum()
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_vjp_corner_200k_sampled_pixels():
    """Full compensation-scale VJP (200k triangles, 512^2, 16 spp, depth 4) on the GPU with
    a cotangent on 24 random clean pixels; the oracle differentiates the same pixels."""
    w = synth.corner_200k()
    w.proj_image = synth.blob_image(512, 512, 77)
    sc = O.Scene(w)
    rng = np.random.default_rng(4)
    px = rng.choice(512 * 512, 48, replace=False)
    m = O.render(sc, pixels=px, want=("margin_clip",))["margin_clip"]
    px = px[(m >= 1).all(axis=1)][:24]
    assert len(px) >= 20
    G = np.zeros((512 * 512, 3))
    G[px] = rng.normal(size=(len(px), 3))
    G = G.reshape(512, 512, 3)
    ref = O.render_vjp(sc, G, pixels=px)
    run = GpuRun(w)
    for mode in ("own", "retrace"):
        gpu = run_vjp(run, G, mode=mode)
        compare_grads(gpu, ref, keys=("Ip", "albedo", "roughness", "specular", "crf_gamma", "white_balance"))


def test_vjp_headline_step_sampled_pixels():
    """The benchmark's step at full size (50k triangles, camera and projector 256^2, 64 spp,
    depth 4, device-built SAH tree): a forward keeping per-sample radiance and path records,
    then the VJP replaying them (binned map flush), with a cotangent on 24 random clean
    pixels and zero elsewhere; the oracle differentiates the same pixels."""
    from paper_2503_12174_amd import dpcs
    w = synth.corner_50k()
    sc = O.Scene(w)
    rng = np.random.default_rng(6)
    px = rng.choice(256 * 256, 48, replace=False)
    m = O.render(sc, pixels=px, want=("margin_clip",))["margin_clip"]
    px = px[(m >= 1).all(axis=1)][:24]
    assert len(px) >= 20
    G = np.zeros((256 * 256, 3))
    G[px] = rng.normal(size=(len(px), 3))
    G = G.reshape(256, 256, 3)
    ref = O.render_vjp(sc, G, pixels=px)
    run = GpuRun(w, scene=dpcs.Scene(ctx(), w.mesh, bvh="sah"))
    compare_grads(run_vjp(run, G, mode="records"), ref)


def test_overlapped_shadow_rays_give_the_serial_results():
    """Full-size waves run a depth's shadow rays on a second stream beside the next depth's
    closest hit; with profiling on every launch stays on one stream.  Forward (image,
    per-sample radiance, path records) and VJP in all three replay modes: bit-identical."""
    from paper_2503_12174_amd import dpcs
    w = synth.corner_50k(spp=32)   # 256^2 x 32 spp: 2^21 paths per wave
    w.env = np.array([0.03, 0.02, 0.04])   # both shadow queues
    run = GpuRun(w, scene=dpcs.Scene(ctx(), w.mesh, bvh="sah"))
    G = np.random.default_rng(3).normal(size=(256, 256, 3))
    res = {}
    try:
        for mode in (0, 1):
            ctx().set_profiling(mode)
            out = run.render()
            res[mode] = dict(img=out["Ic"], L=out["L"], hits=out["hits"],
                             **{m: run_vjp(run, G, mode=m) for m in VJP_MODES})
            ctx().profile()
    finally:
        ctx().set_profiling(0)
    for k in ("img", "L", "hits"):
        np.testing.assert_array_equal(res[0][k], res[1][k], err_msg=k)
    for m in VJP_MODES:
        for name, v in res[1][m].items():
            np.testing.assert_array_equal(res[0][m][name], v, err_msg=f"{m} {name}")


def test_vjp_rejects_bad_arguments():
    import torch
    from paper_2503_12174_amd import dpcs
    w = synth.quad_cube()
    run = GpuRun(w)
    with pytest.raises(dpcs.DpcsError):
        dpcs.dpcs_render_vjp(run.c, run.scene, run.params, run.proj, None)
    rec = torch.zeros((64, 64, w.spp, w.max_depth), dtype=torch.int32, device="cuda")
    G = torch.zeros((64, 64, 3), device="cuda")
    with pytest.raises(dpcs.DpcsError, match="sample_radiance"):   # records without their radiance
        dpcs.dpcs_render_vjp(run.c, run.scene, run.params, run.proj, G, path_records=rec,
                             d_albedo=torch.zeros_like(run.albedo))
    run_vjp(run, np.zeros((64, 64, 3)))   # still usable


def test_path_records_match_hits():
    """Record words name the leaf hit at each vertex: escaped vertices (hit -1) are 0,
    vertices on a surface are nonzero, and the forward image is unchanged by keeping them."""
    import torch
    from paper_2503_12174_amd import dpcs
    w = scenes.c3_ggx(spp=4, seed=5, max_depth=3)
    run = GpuRun(w)
    H, W = w.camera.height, w.camera.width
    hp = torch.full((H, W, w.spp, w.max_depth), -2, dtype=torch.int32, device="cuda")
    rec = torch.zeros((H, W, w.spp, w.max_depth), dtype=torch.int32, device="cuda")
    a = torch.zeros((H, W, 3), device="cuda")
    b = torch.zeros((H, W, 3), device="cuda")
    dpcs.dpcs_render(run.c, run.scene, run.params, run.proj, a, hit_prims=hp)
    dpcs.dpcs_render(run.c, run.scene, run.params, run.proj, b, path_records=rec)
    run.c.synchronize()
    hp, rec = hp.cpu().numpy(), rec.cpu().numpy().view(np.uint32)
    leaf = rec & np.uint32(0x3FFFFFFF)
    assert (leaf[hp == -1] == 0).all()
    assert (leaf[hp >= 0] > 0).all()
    assert ((rec[hp == -1] >> np.uint32(30)) == 0).all()   # no shadow rays from an escaped vertex
    assert (rec[hp >= 0] >> np.uint32(31)).any()           # some projector shadow rays are unoccluded
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_vjp_unbinned_large_maps():
    """BRDF maps and projector image above 1024^2 are not binned: every replay mode
    scatters their cotangents with wave-aggregated atomics instead."""
    import math
    w = scenes.c3_ggx(spp=4, seed=11, max_depth=3)
    w.albedo, w.roughness, w.specular = synth.ggx_textures(909, 1040)
    ang = math.radians(30.0)
    eye_p = (-0.6 * math.sin(ang), 0.0, 0.6 * math.cos(ang))
    w.projector = synth.pinhole(eye_p, (0, 0, 0), 60.0, 1040, 1040, up=(0, 1, 0))
    w.proj_image = np.random.default_rng(910).uniform(0, 1, (1040, 1040, 3)).astype(np.float32)
    sc = O.Scene(w)
    G = _clean_cotangent(w, 7, sc)
    ref = O.render_vjp(sc, G)
    run = GpuRun(w)
    for mode in VJP_MODES:
        compare_grads(run_vjp(run, G, mode=mode), ref)
