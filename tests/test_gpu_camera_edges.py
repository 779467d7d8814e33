"""GPU boundary part of the camera-pose gradient (R_c, t_c of theta, Sec. 3.2) at the images
of mesh edges, through the C ABI: against the oracle on the same edge points and random
numbers, against the exact pixel-coverage gradient, over several launch waves, and its
argument checks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes
from .gpu_util import GpuRun, run_vjp
from .test_gpu_camera import _clean_cotangent
from .test_oracle_pins_camera_edges import (BACK, E1, SQUARE, _cam, _emissive, _exact_gradient, _square_image,
                                            _with_degenerate_faces, _workload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    O.build(force=False)


def _cam_vec(g):
    return np.concatenate([np.ravel(g["camera_R"]), np.ravel(g["camera_t"])])


def _box_scene():
    lo, hi = np.array([-0.3, -0.25, 0.0]), np.array([0.25, 0.3, 0.45])
    box = synth.box_mesh(lo, hi)
    box.emission = np.repeat(np.random.default_rng(7).uniform(0.2, 1.0, (6, 3)), 2, axis=0).astype(np.float32)
    return _workload(box, _cam(eye=(0.9, 0.7, 1.6), target=(0.0, 0.0, 0.2), fov=45.0))


def _scene(name):
    if name == "emissive square":
        return _workload(_emissive(SQUARE, E1), _cam())
    if name == "occluded squares":
        return _workload(synth._merge([_emissive(SQUARE, E1), _emissive(BACK, np.array([0.2, 0.6, 0.9]))]), _cam())
    if name == "closed box":
        return _box_scene()
    if name == "lambert square, depth 2":
        return _workload(synth.quad_mesh(SQUARE), _cam(), albedo=0.6, max_depth=2)
    if name == "faces of no area":
        return _workload(_with_degenerate_faces(_emissive(SQUARE, E1)), _cam())
    # quad + cube under the projector and the environment: textured GGX, occlusion,
    # three vertices, clipping on
    w = scenes.c3_ggx(spp=4, seed=21, max_depth=3)
    w.env = np.array([0.04, 0.06, 0.05])
    return w


@pytest.mark.parametrize("name,density,rtol", [
    ("emissive square", 64, 1e-4), ("occluded squares", 64, 1e-4), ("closed box", 64, 1e-4),
    ("lambert square, depth 2", 64, 1e-4), ("faces of no area", 64, 1e-4), ("quad and cube", 8, 2e-3)])
def test_edge_term_matches_oracle(name, density, rtol):
    """Same edge table, points and random numbers on both sides: the totals agree up to
    FP32 radiance and the odd side path whose decision sits within rounding of a flip."""
    w = _scene(name)
    res = w.camera.width
    if name == "quad and cube":   # the interior part is compared on pixels whose samples are clean
        G = _clean_cotangent(w, 11)
    else:
        G = np.random.default_rng(11).normal(size=(w.camera.height, res, 3))
    # the boundary part alone on each side: with minus without the edges
    ref = _cam_vec(O.render_vjp(O.Scene(w, edge_density=density), G, camera=True)) - \
        _cam_vec(O.render_vjp(O.Scene(w), G, camera=True))
    run = GpuRun(w)
    got = _cam_vec(run_vjp(run, G, mode="records", camera=True, edge_density=density)) - \
        _cam_vec(run_vjp(run, G, mode="records", camera=True))
    scale = np.abs(ref).max()
    assert scale > 1e-3
    err = np.abs(got - ref).max() / scale
    print(f"{name}: boundary part {scale:.3e}, error relative to it {err:.2e}")
    assert err <= rtol, (got, ref)


def test_edge_term_matches_exact_coverage():
    """Independent of the oracle: the emissive square's gradient from exact pixel coverage."""
    w = _workload(_emissive(SQUARE, E1), _cam())
    G = np.random.default_rng(3).normal(size=(24, 24, 3))
    exact = _exact_gradient(_square_image, w.camera, G)
    got = _cam_vec(run_vjp(GpuRun(w), G, mode="own", camera=True, edge_density=1024))
    np.testing.assert_allclose(got, exact, rtol=0, atol=2e-2 * np.abs(exact).max())


def test_edge_term_over_many_waves():
    """A small path capacity cuts the edge points into many launch waves (own queues for
    them, a ragged last wave): the same gradient as one wave."""
    w = _workload(synth._merge([_emissive(SQUARE, E1), _emissive(BACK, np.array([0.2, 0.6, 0.9]))]), _cam())
    G = np.random.default_rng(12).normal(size=(24, 24, 3))
    one = _cam_vec(run_vjp(GpuRun(w), G, mode="records", camera=True, edge_density=256))
    try:
        many = _cam_vec(run_vjp(GpuRun(w, capacity=3000), G, mode="records", camera=True, edge_density=256))
    finally:
        GpuRun(w, capacity=1 << 22)   # the shared context's default again
    np.testing.assert_allclose(many, one, rtol=0, atol=1e-5 * np.abs(one).max())


def test_edge_term_is_deterministic():
    w = _box_scene()
    G = np.random.default_rng(13).normal(size=(24, 24, 3))
    run = GpuRun(w)
    a = _cam_vec(run_vjp(run, G, mode="own", camera=True, edge_density=32))
    b = _cam_vec(run_vjp(run, G, mode="own", camera=True, edge_density=32))
    np.testing.assert_array_equal(a, b)


def test_edge_table_follows_a_refit():
    """After a refit moves the square, the edge table is rebuilt from the moved vertices."""
    import torch
    w = _workload(_emissive(SQUARE, E1), _cam())
    run = GpuRun(w)
    G = np.random.default_rng(14).normal(size=(24, 24, 3))
    run_vjp(run, G, mode="own", camera=True, edge_density=64)   # builds the table
    moved = np.asarray(SQUARE, np.float32) + np.array([0.05, -0.04, 0.1], np.float32)
    run.scene.refit(torch.as_tensor(moved).cuda())
    got = _cam_vec(run_vjp(run, G, mode="own", camera=True, edge_density=64))
    wm = _workload(_emissive([tuple(p) for p in moved], E1), _cam())
    ref = _cam_vec(O.render_vjp(O.Scene(wm, edge_density=64), G, camera=True))
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()


def test_edge_density_argument_checks():
    import torch
    from paper_2503_12174_amd import dpcs
    w = _workload(_emissive(SQUARE, E1), _cam())
    run = GpuRun(w)
    g = torch.zeros((24, 24, 3), device="cuda")
    d = torch.zeros(12, device="cuda")
    with pytest.raises(dpcs.DpcsError, match="INVALID"):
        dpcs.dpcs_render_vjp(run.c, run.scene, run.params, run.proj, g, camera_edge_density=4.0)
    with pytest.raises(dpcs.DpcsError, match="INVALID"):
        dpcs.dpcs_render_vjp(run.c, run.scene, run.params, run.proj, g, d_camera=d, camera_edge_density=-1.0)
    with pytest.raises(dpcs.DpcsError, match="INVALID"):
        dpcs.dpcs_render_vjp(run.c, run.scene, run.params, run.proj, g, d_camera=d, camera_edge_density=float("nan"))


def test_refinement_of_an_emissive_box_needs_the_boundary_part():
    """Every surface of the box only emits, so the pose gradient's interior part is zero and
    only its edges tell where the camera is: refine_camera recovers a pose 0.6 degrees and
    1 cm off with the boundary part, and does not move without it."""
    import copy

    import torch
    from paper_2503_12174_amd import dpcs, drivers
    from .gpu_util import ctx
    w = _box_scene()
    w.camera = synth.pinhole((0.9, 0.7, 1.6), (0.0, 0.0, 0.2), 45.0, 48, 48, up=(0, 1, 0))
    run = GpuRun(w)
    truth = copy.copy(w)
    truth.spp, truth.seed = 16, 1000
    target = torch.zeros((48, 48, 3), device="cuda")
    dpcs.dpcs_render(ctx(), run.scene, dpcs.params_from(truth, run.albedo, run.rough, run.spec), run.proj, target)
    omega0, dt0 = np.array([0.006, -0.008, 0.004]), np.array([0.01, -0.006, 0.008])
    pose0 = drivers.pose_from(torch.tensor(omega0), torch.tensor(dt0), w.camera.R, w.camera.t).numpy()
    start = copy.copy(w)
    start.camera = synth.Pinhole(w.camera.K, pose0[:9].reshape(3, 3), pose0[9:], 48, 48)
    ang = lambda A: np.degrees(np.arccos(np.clip((np.trace(A @ np.asarray(w.camera.R).T) - 1) / 2, -1, 1)))
    before = (ang(pose0[:9].reshape(3, 3)), np.linalg.norm(pose0[9:] - w.camera.t))
    res = {}
    for dens in (0.0, 16.0):
        (R, t), losses = drivers.refine_camera(ctx(), run.scene, start, [run.proj], [target], run.albedo, run.rough,
                                               run.spec, steps=60, lr=1.5e-3, edge_density=dens)
        res[dens] = ((ang(R), np.linalg.norm(t - w.camera.t)), losses)
        print(f"edge density {dens}: pose error {res[dens][0][0]:.3f} deg {res[dens][0][1] * 100:.2f} cm "
              f"(from {before[0]:.3f} deg {before[1] * 100:.2f} cm); loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    (a0, t0), _ = res[0.0]
    assert abs(a0 - before[0]) < 1e-3 * before[0] and abs(t0 - before[1]) < 1e-3 * before[1]
    (a1, t1), losses = res[16.0]
    assert a1 < 0.5 * before[0] and t1 < 0.5 * before[1]
    # (the loss keeps the Monte Carlo noise of 4 against 16 samples per pixel at the edges)
    assert np.mean(losses[-5:]) < 0.8 * np.mean(losses[:3])
