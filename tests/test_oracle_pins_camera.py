"""Pins of the oracle's camera-pose gradient (R_c and t_c of theta, Sec. 3.2).

The oracle differentiates the camera vertex's radiance w.r.t. the 12 entries of (R, t)
with the forward's decisions, sampled directions and later path factors held fixed (the
interior part of the gradient; reading in the design notes).  On the scenes below holding
them fixed is exact, so central differences of the whole rendered image over the pose must
equal the VJP:
  * a plane seen and lit from above, textured GGX, projector and environment next events,
    one vertex -- nothing occludes and the environment direction is sampled about the
    fixed geometric normal;
  * the same plane with a normal map (the shading normal moves with the hit point; the
    environment direction is sampled about the geometric normal);
  * a textured Lambert floor under an emitting black ceiling, two vertices -- the bounce
    leaves in a fixed direction (cosine sampling about the fixed normal) and the ceiling
    returns the same radiance wherever it lands.
"""
import copy

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes

F32 = np.float32


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _textures(rng, n=32):
    alb = rng.uniform(0.2, 0.9, (n, n, 3)).astype(F32)
    rough = rng.uniform(0.2, 0.8, (n, n)).astype(F32)
    spec = rng.uniform(0.2, 1.0, (n, n)).astype(F32)
    return alb, rough, spec


def _proj_image(rng, n=24):
    yy, xx = np.mgrid[0:n, 0:n] / (n - 1.0)
    ramp = np.stack([0.2 + 0.7 * xx, 0.3 + 0.5 * yy, 0.6 - 0.3 * xx * yy], -1)
    return np.clip(ramp + rng.uniform(-0.1, 0.1, (n, n, 3)), 0.0, 1.0).astype(F32)


def lit_plane(normal_map=False, spp=3, res=20):
    """The plane z = 0 under a wide projector and a camera, random GGX maps, a ramp-plus-noise
    projector image, environment on, one vertex."""
    rng = np.random.default_rng(901)
    w = scenes.plane_workload(proj_eye=(0.05, -0.1, 1.0), cam_eye=(0.3, 0.2, 1.2), res=res, pres=24,
                              brdf=synth.GGX, proj_fov=110.0, cam_fov=45.0, spp=spp, max_depth=1, seed=23)
    w.albedo, w.roughness, w.specular = _textures(rng)
    w.proj_image = _proj_image(rng)
    w.env = np.array([0.3, 0.25, 0.2])
    w.crf_gamma = np.array([0.8, 0.9, 1.1])
    if normal_map:
        n = w.albedo.shape[0]
        t = np.stack([rng.uniform(-0.4, 0.4, (n, n)), rng.uniform(-0.4, 0.4, (n, n)), np.ones((n, n))], -1)
        t /= np.linalg.norm(t, axis=-1, keepdims=True)
        w.normal_map = ((t + 1) / 2).astype(F32)
    return w


def floor_under_glowing_ceiling(spp=3, res=20):
    """A Lambert floor z = 0 (random albedo on the left half of the map) under a large black
    ceiling z = 1.5 (right half of the map, albedo 0) that emits 0.7; projector and camera in
    between looking down; two vertices, environment off."""
    rng = np.random.default_rng(902)
    floor = synth.quad_mesh([(-2, -2, 0.0), (2, -2, 0.0), (2, 2, 0.0), (-2, 2, 0.0)], uv_rect=(0.0, 0.0, 0.5, 1.0))
    ceil = synth.quad_mesh([(-30, -30, 1.5), (-30, 30, 1.5), (30, 30, 1.5), (30, -30, 1.5)],
                           uv_rect=(0.5, 0.0, 1.0, 1.0))
    ceil.emission = np.full((ceil.num_triangles, 3), 0.7, F32)
    mesh = synth._merge([floor, ceil])
    alb = np.zeros((16, 32, 3), F32)
    alb[:, :16] = rng.uniform(0.2, 0.9, (16, 16, 3))
    camera = synth.pinhole((0.3, 0.2, 1.2), (0, 0, 0), 45.0, res, res, up=(0, 1, 0))
    projector = synth.pinhole((0.05, -0.1, 1.0), (0, 0, 0), 110.0, 24, 24, up=(0, 1, 0))
    return synth.Workload("floor under a glowing ceiling", mesh, camera, projector, synth.LAMBERT, alb,
                          np.full((16, 32), 0.5, F32), np.full((16, 32), 0.5, F32), _proj_image(rng),
                          prf_gamma=np.full(3, 2.2), prf_gain=1.3, crf_gamma=np.ones(3), white_balance=np.ones(3),
                          clip=False, spp=spp, max_depth=2, seed=29)


def _posed(w, pose):
    v = copy.copy(w)
    c = w.camera
    v.camera = synth.Pinhole(c.K, pose[:9].reshape(3, 3), pose[9:], c.width, c.height)
    return v


def _check(w, h=1e-6, rel=1e-4, **scene_kw):
    res = w.camera.width
    G = np.random.default_rng(5).normal(size=(res, res, 3))
    grad = O.render_vjp(O.Scene(w, **scene_kw), G, camera=True)
    ad = np.concatenate([grad["camera_R"].ravel(), grad["camera_t"]])
    pose = np.concatenate([np.ravel(w.camera.R), np.ravel(w.camera.t)]).astype(np.float64)

    def loss(p):
        return float((O.render(O.Scene(_posed(w, p), **scene_kw), want=("Ic",))["Ic"].reshape(G.shape) * G).sum())

    fd = np.zeros(12)
    for e in range(12):
        d = np.zeros(12)
        d[e] = h
        fd[e] = (loss(pose + d) - loss(pose - d)) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 1e-3
    np.testing.assert_allclose(ad, fd, rtol=rel, atol=rel * scale)
    return ad


def test_camera_pose_gradient_on_a_lit_plane():
    _check(lit_plane())


def test_camera_pose_gradient_through_a_normal_map():
    """The environment direction is sampled about the geometric normal (a flat sampling
    map), so only the evaluation moves with the shading normal."""
    w = lit_plane(normal_map=True)
    flat = np.zeros_like(w.normal_map, dtype=np.float64)
    flat[..., :2], flat[..., 2] = 0.5, 1.0
    _check(w, normal_sample=flat)


def test_camera_pose_gradient_through_the_bounce():
    ad = _check(floor_under_glowing_ceiling())
    # the bounce term carries gradient: without the ceiling's radiance it changes
    w = floor_under_glowing_ceiling()
    w.mesh.emission[:] = 0.0
    res = w.camera.width
    G = np.random.default_rng(5).normal(size=(res, res, 3))
    dark = O.render_vjp(O.Scene(w), G, camera=True)
    assert np.abs(ad - np.concatenate([dark["camera_R"].ravel(), dark["camera_t"]])).max() > 1e-3 * np.abs(ad).max()


def test_camera_pose_gradient_is_zero_for_a_uniform_view():
    """A Lambert plane of constant albedo under constant environment light only (projector
    dark): every camera sample sees the same radiance, so moving the camera changes
    nothing."""
    w = scenes.plane_workload(res=12, const_image=0.0, albedo=0.6, max_depth=1, spp=2)
    w.env = np.array([0.5, 0.4, 0.3])
    res = w.camera.width
    G = np.random.default_rng(1).normal(size=(res, res, 3))
    g = O.render_vjp(O.Scene(w), G, camera=True)
    assert np.abs(g["camera_R"]).max() < 1e-6 and np.abs(g["camera_t"]).max() < 1e-6
