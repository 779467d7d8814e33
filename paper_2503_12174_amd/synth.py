"""Seeded synthetic inputs: meshes, textures, projector images, camera/projector poses.

This module builds inputs only. It holds none of the rendering method's arithmetic
(no projection, shading, response functions or sampling); both the GPU library
and the CPU oracle consume the arrays it returns.

The paper measures on real captured setups that are not available here
(Sec. 4: camera 640x360, projector 800x600, 16 spp training). The generators
below stand in for them with scenes of the same kind: a projection surface
with interreflection (a folded corner), occluders casting projector shadows,
textured BRDF maps and natural-image-like projector patterns.

Conventions shared by every consumer:
  * vertices: float32 [V, 3]; triangles: int32 [T, 3]; per-corner UVs float32 [T, 3, 2]
  * textures: float32, row-major, [H, W, C]; row index follows v, column follows u
  * pinhole devices: K (3x3), R (3x3), t (3); a world point x maps to device
    coordinates R x + t (OpenCV axes: +x right, +y down, +z forward)
  * images: float32 [H, W, 3], HWC row-major
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


# ----------------------------------------------------------------------------
# poses / intrinsics (stand-ins for the calibration the paper takes as given)
# ----------------------------------------------------------------------------

def intrinsics(fov_deg: float, width: int, height: int) -> np.ndarray:
    """Square-pixel pinhole intrinsics with a horizontal field of view."""
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return np.array([[f, 0.0, width / 2.0], [0.0, f, height / 2.0], [0.0, 0.0, 1.0]])


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World->device rotation R and translation t for a device at `eye` looking at `target`."""
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    return R, t


@dataclass
class Pinhole:
    K: np.ndarray
    R: np.ndarray
    t: np.ndarray
    width: int
    height: int


def pinhole(eye, target, fov_deg, width, height, up=(0.0, 0.0, 1.0)) -> Pinhole:
    R, t = look_at(eye, target, up)
    K = intrinsics(fov_deg, width, height)
    return Pinhole(K, R, t, int(width), int(height))


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    vertices: np.ndarray            # float32 [V,3]
    triangles: np.ndarray           # int32 [T,3]
    corner_uvs: np.ndarray          # float32 [T,3,2]
    emission: np.ndarray | None = None   # float32 [T,3] (test scenes only)

    @property
    def num_triangles(self) -> int:
        return int(self.triangles.shape[0])


def _merge(parts):
    vs, fs, uvs, ems = [], [], [], []
    off = 0
    have_em = any(p.emission is not None for p in parts)
    for p in parts:
        vs.append(p.vertices)
        fs.append(p.triangles + off)
        uvs.append(p.corner_uvs)
        if have_em:
            ems.append(p.emission if p.emission is not None
                       else np.zeros((p.num_triangles, 3), F32))
        off += p.vertices.shape[0]
    return Mesh(np.concatenate(vs).astype(F32), np.concatenate(fs).astype(np.int32),
                np.concatenate(uvs).astype(F32),
                np.concatenate(ems).astype(F32) if have_em else None)


def quad_mesh(corners, uv_rect=(0.0, 0.0, 1.0, 1.0)) -> Mesh:
    """Two triangles over 4 corners given counter-clockwise (c0,c1,c2,c3)."""
    c = np.asarray(corners, dtype=np.float64)
    u0, v0, u1, v1 = uv_rect
    uv = np.array([[u0, v0], [u1, v0], [u1, v1], [u0, v1]])
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return Mesh(c.astype(F32), tris, uv[tris].astype(F32))


def box_mesh(lo, hi, uv_rect=(0.0, 0.0, 1.0, 1.0), inward=False) -> Mesh:
    """Axis-aligned box, 12 triangles, every face mapped to uv_rect."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    faces = [
        [(x0, y0, z0), (x0, y1, z0), (x1, y1, z0), (x1, y0, z0)],  # z-
        [(x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)],  # z+
        [(x0, y0, z0), (x1, y0, z0), (x1, y0, z1), (x0, y0, z1)],  # y-
        [(x0, y1, z0), (x0, y1, z1), (x1, y1, z1), (x1, y1, z0)],  # y+
        [(x0, y0, z0), (x0, y0, z1), (x0, y1, z1), (x0, y1, z0)],  # x-
        [(x1, y0, z0), (x1, y1, z0), (x1, y1, z1), (x1, y0, z1)],  # x+
    ]
    parts = []
    for f in faces:
        if inward:
            f = f[::-1]
        parts.append(quad_mesh(f, uv_rect))
    return _merge(parts)


def plane_grid(n: int, origin, axis_u, axis_v, size_u: float, size_v: float,
               uv_rect=(0.0, 0.0, 1.0, 1.0), height=None) -> Mesh:
    """n x n quad grid spanning origin + s*axis_u + r*axis_v, s in [0,size_u], r in [0,size_v].

    `height(s, r)` (optional) returns a displacement along axis_u x axis_v.
    """
    origin = np.asarray(origin, np.float64)
    au = np.asarray(axis_u, np.float64)
    av = np.asarray(axis_v, np.float64)
    normal = np.cross(au, av)
    s = np.linspace(0.0, size_u, n + 1)
    r = np.linspace(0.0, size_v, n + 1)
    S, Rr = np.meshgrid(s, r, indexing="ij")
    P = origin + S[..., None] * au + Rr[..., None] * av
    if height is not None:
        P = P + height(S, Rr)[..., None] * normal
    V = P.reshape(-1, 3)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    u0, v0, u1, v1 = uv_rect
    U = u0 + (u1 - u0) * (S / size_u)
    W = v0 + (v1 - v0) * (Rr / size_v)
    uvv = np.stack([U, W], -1).reshape(-1, 2)
    return Mesh(V.astype(F32), tris.astype(np.int32), uvv[tris].astype(F32))


# improved gradient noise (Perlin, "Improving Noise", SIGGRAPH 2002), 3-D form
_GRAD3 = np.array([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0],
                   [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
                   [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1],
                   [1, 1, 0], [-1, 1, 0], [0, -1, 1], [0, -1, -1]], np.float64)


def perlin3(x, y, z, perm):
    p = np.concatenate([perm, perm])
    xi = np.floor(x).astype(np.int64)
    yi = np.floor(y).astype(np.int64)
    zi = np.floor(z).astype(np.int64)
    xf, yf, zf = x - xi, y - yi, z - zi
    xi &= 255
    yi &= 255
    zi &= 255

    def fade(t):
        return t * t * t * (t * (t * 6 - 15) + 10)

    u, v, w = fade(xf), fade(yf), fade(zf)

    def g(h, dx, dy, dz):
        gv = _GRAD3[h & 15]
        return gv[..., 0] * dx + gv[..., 1] * dy + gv[..., 2] * dz

    A = p[xi] + yi
    AA = p[A] + zi
    AB = p[A + 1] + zi
    B = p[xi + 1] + yi
    BA = p[B] + zi
    BB = p[B + 1] + zi

    def lerp(t, a, b):
        return a + t * (b - a)

    x1 = lerp(u, g(p[AA], xf, yf, zf), g(p[BA], xf - 1, yf, zf))
    x2 = lerp(u, g(p[AB], xf, yf - 1, zf), g(p[BB], xf - 1, yf - 1, zf))
    y1 = lerp(v, x1, x2)
    x3 = lerp(u, g(p[AA + 1], xf, yf, zf - 1), g(p[BA + 1], xf - 1, yf, zf - 1))
    x4 = lerp(u, g(p[AB + 1], xf, yf - 1, zf - 1), g(p[BB + 1], xf - 1, yf - 1, zf - 1))
    y2 = lerp(v, x3, x4)
    return lerp(w, y1, y2)


def _boxes(rng, count):
    boxes = []
    while len(boxes) < count:
        e = rng.uniform(0.05, 0.12, size=3)
        c = np.array([rng.uniform(0.2, 0.5), rng.uniform(-0.3, 0.3), rng.uniform(0.2, 0.5)])
        lo, hi = c - e / 2, c + e / 2
        ok = True
        for (blo, bhi) in boxes:  # no contact between boxes (1 cm gap)
            if np.all(lo < bhi + 0.01) and np.all(blo < hi + 0.01):
                ok = False
        if ok:
            boxes.append((lo, hi))
    return boxes


def folded_corner(n: int, perlin_seed: int, box_seed: int | None, n_boxes: int = 3,
                  amplitude: float = 0.02, cycles_per_m: float = 4.0, taper: float = 0.02) -> Mesh:
    """Floor (z=0, x in [0,1]) and wall (x=0, z in [0,1]), y in [-0.5,0.5], n x n quads each.

    Displaced along the plane normal by amplitude * noise, tapered to zero within
    `taper` metres of the fold; optional floating box occluders (UV strip [0.9,1]).
    """
    perm = np.random.default_rng(perlin_seed).permutation(256)

    def disp(dist, other, zoff):
        k = np.clip(dist / taper, 0.0, 1.0)
        k = k * k * (3 - 2 * k)
        return amplitude * k * perlin3(dist * cycles_per_m, other * cycles_per_m,
                                       np.full_like(dist, zoff), perm)

    # floor: s along +x, r along +y (normal +z)
    floor = plane_grid(n, (0.0, -0.5, 0.0), (1, 0, 0), (0, 1, 0), 1.0, 1.0,
                       uv_rect=(0.0, 0.0, 0.45, 1.0),
                       height=lambda S, Rr: disp(S, Rr - 0.5, 0.37))
    # wall: s along +y, r along +z (normal +x)
    wall = plane_grid(n, (0.0, -0.5, 0.0), (0, 1, 0), (0, 0, 1), 1.0, 1.0,
                      uv_rect=(0.45, 0.0, 0.9, 1.0),
                      height=lambda S, Rr: disp(Rr, S - 0.5, 0.71))
    # wall UVs: u follows height z, v follows y (swap the grid's uv roles)
    uvw = wall.corner_uvs.copy()
    uvw = np.stack([0.45 + (uvw[..., 1]) * 0.45, (uvw[..., 0] - 0.45) / 0.45], -1).astype(F32)
    wall = Mesh(wall.vertices, wall.triangles, uvw)
    parts = [floor, wall]
    if box_seed is not None and n_boxes > 0:
        for lo, hi in _boxes(np.random.default_rng(box_seed), n_boxes):
            parts.append(box_mesh(lo, hi, uv_rect=(0.9, 0.0, 1.0, 1.0)))
    return _merge(parts)


def quad_and_cube() -> Mesh:
    """1 m^2 quad at z=0 plus a 0.2 m cube resting on it (14 triangles)."""
    quad = quad_mesh([(-0.5, -0.5, 0.0), (0.5, -0.5, 0.0), (0.5, 0.5, 0.0), (-0.5, 0.5, 0.0)])
    cube = box_mesh((0.05, -0.1, 0.0), (0.25, 0.1, 0.2))
    return _merge([quad, cube])


def closed_box(half: float = 0.5, emission=(1.0, 1.0, 1.0)) -> Mesh:
    """Closed cube [-half,half]^3, faces wound inward, uniform emission (white-furnace scene)."""
    m = box_mesh((-half, -half, -half), (half, half, half), inward=True)
    m.emission = np.tile(np.asarray(emission, F32), (m.num_triangles, 1))
    return m


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Geodesic sphere (icosahedron subdivided `level` times), UVs by spherical angles."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts) * radius
    F = np.array(faces, np.int32)
    d = V / radius
    uv = np.stack([0.5 + np.arctan2(d[:, 1], d[:, 0]) / (2 * np.pi), np.arccos(np.clip(d[:, 2], -1, 1)) / np.pi], 1)
    return Mesh(V.astype(F32), F, uv[F].astype(F32))


# ----------------------------------------------------------------------------
# textures / images
# ----------------------------------------------------------------------------

def uniform_texture(rng, h, w, c, lo, hi):
    return rng.uniform(lo, hi, size=(h, w, c)).astype(F32)


def blob_image(h: int, w: int, seed: int, n_blobs: int = 8, noise: float = 0.05,
               lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Natural-image-like field: sum of random Gaussian blobs + uniform noise, clipped."""
    rng = np.random.default_rng(seed)
    ys, xs = np.meshgrid((np.arange(h) + 0.5) / h, (np.arange(w) + 0.5) / w, indexing="ij")
    img = np.zeros((h, w, 3))
    size = max(h, w)
    for _ in range(n_blobs):
        cx, cy = rng.uniform(0, 1, 2)
        sigma = rng.uniform(0.05, 0.3) * size
        amp = rng.uniform(0, 1, 3)
        d2 = ((xs - cx) * w) ** 2 + ((ys - cy) * h) ** 2
        img += np.exp(-d2 / (2 * sigma * sigma))[..., None] * amp
    img /= max(img.max(), 1e-12)
    img += rng.uniform(0, noise, size=img.shape)
    img = np.clip(img, 0.0, 1.0)
    return (lo + (hi - lo) * img).astype(F32)


# ----------------------------------------------------------------------------
# full workloads
# ----------------------------------------------------------------------------

LAMBERT = 0
GGX = 1


@dataclass
class Workload:
    name: str
    mesh: Mesh
    camera: Pinhole
    projector: Pinhole
    brdf: int
    albedo: np.ndarray        # [Ht,Wt,3]
    roughness: np.ndarray     # [Ht,Wt]
    specular: np.ndarray      # [Ht,Wt]
    proj_image: np.ndarray    # [Hp,Wp,3]
    prf_gamma: np.ndarray = field(default_factory=lambda: np.full(3, 2.2))
    prf_gain: float = 1.0
    prf_mix: np.ndarray = field(default_factory=lambda: np.eye(3))
    crf_gamma: np.ndarray = field(default_factory=lambda: np.full(3, 1 / 2.2))
    crf_gain: float = 1.0
    white_balance: np.ndarray = field(default_factory=lambda: np.ones(3))
    env: np.ndarray = field(default_factory=lambda: np.zeros(3))
    clip: bool = True
    clip_k: float = 1.0
    spp: int = 4
    max_depth: int = 3
    seed: int = 0
    sample_offset: int = 0
    metallic: np.ndarray | None = None     # [Ht,Wt] metallic map (GGX), None: 0
    normal_map: np.ndarray | None = None   # [Ht,Wt,3] stored normal map in [0,1], None: none

    def scalars(self):
        return dict(prf_gamma=self.prf_gamma, prf_gain=self.prf_gain, prf_mix=self.prf_mix,
                    crf_gamma=self.crf_gamma, crf_gain=self.crf_gain,
                    white_balance=self.white_balance, env=self.env, clip=self.clip,
                    clip_k=self.clip_k, spp=self.spp, max_depth=self.max_depth, seed=self.seed,
                    sample_offset=self.sample_offset, brdf=self.brdf)


def _f32(a):
    return np.asarray(a, np.float64).astype(F32).astype(np.float64)


def quad_cube(spp: int = 4, max_depth: int = 3, seed: int = 0) -> Workload:
    """Plain forward render at oracle scale: quad + cube, Lambert, 64x64 camera/projector."""
    mesh = quad_and_cube()
    albedo = uniform_texture(np.random.default_rng(101), 64, 64, 3, 0.2, 0.8)
    proj = np.random.default_rng(102).uniform(0, 1, size=(64, 64, 3)).astype(F32)
    ang = math.radians(30.0)
    eye_p = (-0.6 * math.sin(ang), 0.0, 0.6 * math.cos(ang))
    projector = pinhole(eye_p, (0, 0, 0), 60.0, 64, 64, up=(0, 1, 0))
    camera = pinhole((0, 0, 0.8), (0, 0, 0), 60.0, 64, 64, up=(0, 1, 0))
    return Workload("quad+cube 14 tris, cam 64x64, proj 64x64, Lambert, 4 spp, D=3",
                    mesh, camera, projector, LAMBERT, albedo,
                    np.full((64, 64), 0.5, F32), np.zeros((64, 64), F32), proj,
                    white_balance=_f32((1.0, 0.95, 1.05)), spp=spp, max_depth=max_depth, seed=seed)


def ggx_textures(seed: int, size: int):
    rng = np.random.default_rng(seed)
    albedo = uniform_texture(rng, size, size, 3, 0.2, 0.8)
    rough = uniform_texture(rng, size, size, 1, 0.1, 0.9)[..., 0]
    spec = uniform_texture(rng, size, size, 1, 0.0, 1.0)[..., 0]
    return albedo, rough, spec


def corner_50k(spp: int = 64, max_depth: int = 4, seed: int = 0, env: float = 0.0,
            res: int = 256, n_quads: int = 112) -> Workload:
    """Forward at the paper's scale: 50k-triangle displaced folded corner + 3 boxes, GGX."""
    mesh = folded_corner(n_quads, 201, 202)
    albedo, rough, spec = ggx_textures(203, 512)
    camera = pinhole((0.85, 0.0, 0.85), (0.3, 0.0, 0.3), 60.0, res, res)
    projector = pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, 256, 256)
    proj = blob_image(256, 256, 204)
    return Workload(f"folded corner {mesh.num_triangles} tris + 3 boxes, GGX 512^2 textures, "
                    f"cam {res}x{res}, proj 256x256, {spp} spp, D={max_depth}",
                    mesh, camera, projector, GGX, albedo, rough, spec, proj,
                    env=np.full(3, env), spp=spp, max_depth=max_depth, seed=seed)


def corner_capture_res(spp: int = 16, max_depth: int = 4, seed: int = 0) -> Workload:
    """The 50k-triangle corner at the paper's capture resolutions (Sec. 4): camera
    640x360, projector 800x600, 16 spp (its training and relighting sample count)."""
    w = corner_50k(spp=spp, max_depth=max_depth, seed=seed)
    w.camera = pinhole((0.85, 0.0, 0.85), (0.3, 0.0, 0.3), 60.0, 640, 360)
    w.projector = pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, 800, 600)
    w.proj_image = blob_image(600, 800, 205)
    w.name = (f"folded corner {w.mesh.num_triangles} tris + 3 boxes, GGX 512^2 textures, cam 640x360, "
              f"proj 800x600, {spp} spp, D={max_depth}")
    return w


def fit_truth(seed: int = 301):
    """Hidden ground truth for the scene-parameter fit (textures 64^2, PRF/CRF, mixing, WB)."""
    rng = np.random.default_rng(seed)
    albedo = uniform_texture(rng, 64, 64, 3, 0.2, 0.8)
    rough = uniform_texture(rng, 64, 64, 1, 0.1, 0.9)[..., 0]
    spec = uniform_texture(rng, 64, 64, 1, 0.0, 1.0)[..., 0]
    prf_gamma = _f32(rng.uniform(1.8, 2.6, 3))
    crf_gamma = _f32(1.0 / rng.uniform(1.8, 2.6, 3))
    mix = _f32(np.eye(3) + rng.uniform(-0.1, 0.1, (3, 3)))
    wb = _f32(rng.uniform(0.9, 1.1, 3))
    return dict(albedo=albedo, roughness=rough, specular=spec, prf_gamma=prf_gamma,
                crf_gamma=crf_gamma, prf_mix=mix, white_balance=wb)


def fit_scene(spp: int = 32, seed: int = 0) -> Workload:
    """The quad-and-cube scene with GGX maps at the fit's initial guess."""
    w = quad_cube(spp=spp, seed=seed)
    w.name = "quad+cube 14 tris, GGX 64^2 maps, fit step (8 images, 32 spp fwd+VJP)"
    w.brdf = GGX
    w.albedo = np.full((64, 64, 3), 0.5, F32)
    w.roughness = np.full((64, 64), 0.5, F32)
    w.specular = np.full((64, 64), 0.5, F32)
    w.white_balance = np.ones(3)
    return w


def fit_images(step: int, count: int = 8):
    rng = np.random.default_rng(3000 + step)
    return rng.uniform(0, 1, size=(count, 64, 64, 3)).astype(F32)


def corner_200k(spp: int = 16, max_depth: int = 4, seed: int = 0, n_quads: int = 224,
            res: int = 512) -> Workload:
    """Compensation scale: 200k-triangle folded corner, 512^2 GGX maps, 512^2 camera/projector."""
    mesh = folded_corner(n_quads, 401, 402)
    albedo, rough, spec = ggx_textures(401, 512)
    camera = pinhole((0.85, 0.0, 0.85), (0.3, 0.0, 0.3), 60.0, res, res)
    projector = pinhole((0.85, 0.15, 0.85), (0.3, 0.0, 0.3), 45.0, res, res)
    proj = np.full((res, res, 3), 0.5, F32)
    return Workload(f"folded corner {mesh.num_triangles} tris + 3 boxes, GGX 512^2 maps, "
                    f"cam {res}x{res}, proj {res}x{res}, {spp} spp, D={max_depth}",
                    mesh, camera, projector, GGX, albedo, rough, spec, proj,
                    spp=spp, max_depth=max_depth, seed=seed)


def compensation_target(res: int = 512):
    return blob_image(res, res, 402, lo=0.1, hi=0.9)


SERVING_QUADS = (50, 112, 224, 354)


def serving_scenes():
    """Four resident corners of 10,000 / 50,176 / 200,704 / 501,264 triangles (+36 box tris)."""
    return [folded_corner(n, 510 + i, 520 + i) for i, n in enumerate(SERVING_QUADS)]


def serving_requests(count: int, seed: int = 501, rate: float = 50.0):
    """Poisson arrival times and request shapes for the serving workload."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    out = []
    for k in range(count):
        res = int(rng.choice([128, 256, 512]))
        out.append(dict(arrival=float(arrivals[k]), scene=int(rng.integers(0, 4)), res=res,
                        spp=int(rng.choice([16, 64, 256])), depth=4,
                        compensation=bool(rng.integers(0, 2)), image_seed=int(rng.integers(0, 2**31))))
    return out
