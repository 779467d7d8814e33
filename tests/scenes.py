"""Small test scenes built from the seeded generators (inputs only, no rendering arithmetic)."""
from __future__ import annotations

import copy
import math

import numpy as np

from paper_2503_12174_amd import synth

F32 = np.float32


def plane_workload(proj_eye=(0.0, 0.0, 1.0), cam_eye=(0.3, 0.2, 1.2), half=2.0, res=32, pres=32,
                   const_image=0.6, albedo=0.5, tex=None, max_depth=1, spp=4, brdf=synth.LAMBERT,
                   proj_fov=50.0, cam_fov=50.0, seed=7):
    """A single large quad z=0 (UV = affine in x,y), a projector and a camera above it."""
    mesh = synth.quad_mesh([(-half, -half, 0.0), (half, -half, 0.0), (half, half, 0.0), (-half, half, 0.0)])
    projector = synth.pinhole(proj_eye, (0, 0, 0), proj_fov, pres, pres, up=(0, 1, 0))
    camera = synth.pinhole(cam_eye, (0, 0, 0), cam_fov, res, res, up=(0, 1, 0))
    if tex is None:
        tex = np.full((8, 8, 3), albedo, F32)
    th, tw = tex.shape[:2]
    img = np.full((pres, pres, 3), const_image, F32)
    return synth.Workload("test plane", mesh, camera, projector, brdf, tex,
                          np.full((th, tw), 0.5, F32), np.full((th, tw), 0.5, F32), img,
                          prf_gamma=np.full(3, 2.2), prf_gain=1.7, crf_gamma=np.ones(3),
                          white_balance=np.ones(3), clip=False, spp=spp, max_depth=max_depth, seed=seed)


def c1_direct(spp=4, seed=3, const_image=0.8, albedo=0.6):
    """Quad-and-cube geometry, direct light only, constant albedo and projector image."""
    w = synth.quad_cube(spp=spp, max_depth=1, seed=seed)
    w.albedo = np.full_like(w.albedo, albedo)
    w.proj_image = np.full_like(w.proj_image, const_image)
    w.clip = False
    w.crf_gamma = np.ones(3)
    w.white_balance = np.ones(3)
    return w


def furnace_workload(rho=0.7, max_depth=4, spp=4, res=16, le=1.0):
    """Closed emissive Lambertian box with the camera and the projector inside; projector dark."""
    mesh = synth.closed_box(0.5, emission=(le, le, le))
    camera = synth.pinhole((0.1, -0.05, 0.02), (0.4, 0.3, -0.2), 80.0, res, res)
    projector = synth.pinhole((-0.2, 0.1, 0.1), (0.3, 0.0, 0.0), 60.0, 8, 8)
    tex = np.full((4, 4, 3), rho, F32)
    return synth.Workload("furnace", mesh, camera, projector, synth.LAMBERT, tex,
                          np.full((4, 4), 0.5, F32), np.zeros((4, 4), F32), np.zeros((8, 8, 3), F32),
                          clip=False, spp=spp, max_depth=max_depth, seed=11)


def linear_params(w):
    """Make the map projector image -> camera image linear (gamma 1, gains 1, no clip, dark env)."""
    w = copy.copy(w)
    w.prf_gamma = np.ones(3)
    w.crf_gamma = np.ones(3)
    w.prf_gain = 1.0
    w.crf_gain = 1.0
    w.white_balance = np.ones(3)
    w.prf_mix = np.eye(3)
    w.clip = False
    w.env = np.zeros(3)
    return w


def c3_ggx(spp=4, seed=5, max_depth=3):
    """Quad-and-cube geometry with random GGX maps (64^2) and non-trivial PRF/CRF parameters."""
    w = synth.quad_cube(spp=spp, max_depth=max_depth, seed=seed)
    t = synth.fit_truth(301)
    w.brdf = synth.GGX
    w.albedo, w.roughness, w.specular = t["albedo"], t["roughness"], t["specular"]
    w.prf_gamma, w.crf_gamma, w.prf_mix, w.white_balance = t["prf_gamma"], t["crf_gamma"], t["prf_mix"], t["white_balance"]
    return w


def project(K, R, t, x):
    """Pixel coordinates of world points x (n x 3) under K [R | t] with the perspective divide."""
    p = (np.asarray(R) @ np.asarray(x).T).T + np.asarray(t)
    q = (np.asarray(K) @ p.T).T
    return q[:, :2] / q[:, 2:3], p


def philox_u(seed, pixel, sample, block):
    from oracle import oracle as O
    c = np.array([[pixel, sample, block, 0]], np.uint32)
    x = O.philox(seed, c)[0]
    return (x >> 8).astype(np.float64) * 2.0 ** -24


def deg(a):
    return math.radians(a)
