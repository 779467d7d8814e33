"""Pins of the boundary part of the oracle's camera-pose gradient (R_c, t_c of theta, Sec. 3.2).

A pixel is the integral of the sample radiance over its unit square of image coordinates
(the uniform jitter of the camera samples, Eq. 6).  On scenes whose surfaces only emit
(albedo 0) in front of a constant environment, the radiance is piecewise constant in the
image, so a pixel's value is exactly

    I_p = L_env + sum over visible faces of (E_face - L_env) * area(face image  ∩  pixel),

with the face images clipped by polygon clipping here (Sutherland-Hodgman, shoelace area;
no ray is traced).  Its derivative over the 12 pose entries by central differences is the
exact camera-pose gradient, and the interior part is zero (the radiance does not depend
on where a face is hit), so the oracle's boundary estimate -- stratified points along the
images of the mesh edges, the jump from two paths beside each point -- must converge to
it.  The cases:
  * one emissive square (silhouette edges, a coplanar diagonal that must add nothing);
  * a front square partly hiding a back square (edges hidden behind a surface, edges that
    pass behind another's image);
  * a square whose two triangles emit differently (an emission seam) and a folded strip of
    equal emission (a crease with no jump: nothing may be added);
  * a closed box with a different emission on every face (silhouettes of a solid, creases
    between visible faces, edges hidden behind the solid), and one of a single emission
    without texture seams (only the silhouette jumps);
  * two coplanar triangles folded flat onto one side of their edge;
  * faces of no area (a sliver on a silhouette edge, a repeated corner) that change nothing;
  * a floor that reaches behind the camera (edges clipped at the camera plane);
  * a Lambert square of albedo rho under the environment alone: its radiance is
    rho * L_env exactly (environment next event with cosine sampling, nothing above), so
    the jump comes from path tracing rather than emission; the same with a texture seam
    along its diagonal.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

F32 = np.float32
ENV = np.array([0.1, 0.15, 0.2])


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


# ------------------------------------------------------------------ exact coverage
def clip_half(poly, a, b, c):
    """Part of polygon poly (list of (x, y)) with a x + b y <= c."""
    out = []
    for k in range(len(poly)):
        p, q = poly[k], poly[(k + 1) % len(poly)]
        fp, fq = a * p[0] + b * p[1] - c, a * q[0] + b * q[1] - c
        if fp <= 0:
            out.append(p)
        if fp * fq < 0:
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def clip_convex(poly, conv):
    """poly ∩ conv for a convex polygon conv (either orientation)."""
    s = sum(conv[k][0] * conv[(k + 1) % len(conv)][1] - conv[(k + 1) % len(conv)][0] * conv[k][1]
            for k in range(len(conv)))
    for k in range(len(conv)):
        p, q = conv[k], conv[(k + 1) % len(conv)]
        # inside = left of p->q for a counter-clockwise conv (s > 0)
        a, b = (q[1] - p[1]), -(q[0] - p[0])
        if s < 0:
            a, b = -a, -b
        poly = clip_half(poly, a, b, a * p[0] + b * p[1])
        if not poly:
            break
    return poly


def area(poly):
    if len(poly) < 3:
        return 0.0
    return 0.5 * abs(sum(poly[k][0] * poly[(k + 1) % len(poly)][1] - poly[(k + 1) % len(poly)][0] * poly[k][1]
                         for k in range(len(poly))))


def image_polygon(cam_K, R, t, pts, wmin=1e-6):
    """Image of a planar 3D polygon: clipped to w >= wmin in front of the camera, projected."""
    X = [cam_K @ (R @ np.asarray(p, float) + t) for p in pts]
    kept = []
    for k in range(len(X)):
        p, q = X[k], X[(k + 1) % len(X)]
        if p[2] >= wmin:
            kept.append(p)
        if (p[2] - wmin) * (q[2] - wmin) < 0:
            s = (wmin - p[2]) / (q[2] - p[2])
            kept.append(p + s * (q - p))
    return [(h[0] / h[2], h[1] / h[2]) for h in kept]


def pixel_areas(poly, W, H):
    cov = np.zeros((H, W))
    if len(poly) < 3:
        return cov
    xs, ys = [p[0] for p in poly], [p[1] for p in poly]
    for j in range(max(0, int(np.floor(min(ys)))), min(H, int(np.ceil(max(ys))))):
        for i in range(max(0, int(np.floor(min(xs)))), min(W, int(np.ceil(max(xs))))):
            c = clip_half(clip_half(clip_half(clip_half(poly, 1, 0, i + 1), -1, 0, -i), 0, 1, j + 1), 0, -1, -j)
            cov[j, i] = area(c)
    return cov


# ------------------------------------------------------------------ scenes
def _workload(mesh, cam, albedo=0.0, spp=2, max_depth=1):
    prj = synth.pinhole((0.0, 0.0, 1.0), (0, 0, 0), 50.0, 8, 8, up=(0, 1, 0))
    return synth.Workload("edges", mesh, cam, prj, synth.LAMBERT, np.full((4, 4, 3), albedo, F32),
                          np.full((4, 4), 0.5, F32), np.full((4, 4), 0.5, F32), np.zeros((8, 8, 3), F32),
                          crf_gamma=np.ones(3), white_balance=np.ones(3), env=ENV, clip=False, spp=spp,
                          max_depth=max_depth, seed=3)


def _emissive(corners, e):
    m = synth.quad_mesh(corners)
    m.emission = np.tile(np.asarray(e, F32), (2, 1))
    return m


def _cam(res=24, eye=(0.2, 0.1, 2.0), target=(0.02, -0.03, 0.0), fov=40.0):
    return synth.pinhole(eye, target, fov, res, res, up=(0, 1, 0))


SQUARE = [(-0.3, -0.25, 0.4), (0.35, -0.3, 0.4), (0.3, 0.28, 0.4), (-0.32, 0.3, 0.4)]
BACK = [(-0.05, -0.45, 0.1), (0.55, -0.4, 0.1), (0.5, 0.15, 0.1), (-0.1, 0.1, 0.1)]


def _pose(cam):
    return np.concatenate([np.ravel(cam.R), np.ravel(cam.t)]).astype(np.float64)


def _exact_gradient(image_fn, cam, G, h=1e-6):
    """Central differences over the 12 pose entries of sum(G * image_fn(K, R, t))."""
    p0 = _pose(cam)

    def loss(p):
        return float((image_fn(cam.K, p[:9].reshape(3, 3), p[9:]) * G).sum())

    out = np.zeros(12)
    for e in range(12):
        d = np.zeros(12)
        d[e] = h
        out[e] = (loss(p0 + d) - loss(p0 - d)) / (2 * h)
    return out


def _check(w, image_fn, density, rtol, G=None, seed=1):
    res = w.camera.width
    if G is None:
        G = np.random.default_rng(seed).normal(size=(res, res, 3))
    exact = _exact_gradient(image_fn, w.camera, G)
    b, n = O.camera_boundary(O.Scene(w, edge_density=density), G)
    assert n > 0
    scale = np.abs(exact).max()
    assert scale > 1e-2
    np.testing.assert_allclose(b, exact, rtol=0, atol=rtol * scale)
    return b, exact


# ------------------------------------------------------------------ pins
E1 = np.array([0.8, 0.5, 0.3])


def _square_image(K, R, t, res=24):
    cov = pixel_areas(image_polygon(K, R, t, SQUARE), res, res)
    return ENV + (E1 - ENV) * cov[..., None]


def test_square_silhouette_constant_cotangent():
    """Constant cotangent: the integrand is smooth along each edge, so stratified points
    converge fast."""
    w = _workload(_emissive(SQUARE, E1), _cam())
    G = np.ones((24, 24, 3)) * np.array([0.7, -0.4, 1.1])
    _check(w, _square_image, 16, 1e-3, G=G)


def test_square_silhouette_random_cotangent():
    """Random per-pixel cotangents: the points must land in the right pixels."""
    w = _workload(_emissive(SQUARE, E1), _cam())
    _check(w, _square_image, 1024, 2e-2)


def test_square_boundary_converges():
    """The error of the stratified estimate falls with the density (no bias)."""
    w = _workload(_emissive(SQUARE, E1), _cam())
    G = np.random.default_rng(4).normal(size=(24, 24, 3))
    exact = _exact_gradient(_square_image, w.camera, G)
    errs = [np.abs(O.camera_boundary(O.Scene(w, edge_density=d), G)[0] - exact).max() for d in (4, 64, 2048)]
    assert errs[2] < 0.1 * errs[0]


def test_occluded_edges():
    """A front square hides part of a back square: the back square's edges behind the
    front one must add nothing; the front square's edges over the back one jump between
    the two emissions."""
    EB = np.array([0.2, 0.6, 0.9])
    mesh = synth._merge([_emissive(SQUARE, E1), _emissive(BACK, EB)])
    w = _workload(mesh, _cam())

    def image(K, R, t):
        f = image_polygon(K, R, t, SQUARE)
        b = image_polygon(K, R, t, BACK)
        cf, cb = pixel_areas(f, 24, 24), pixel_areas(b, 24, 24)
        cfb = pixel_areas(clip_convex(b, f), 24, 24)
        return ENV + (E1 - ENV) * cf[..., None] + (EB - ENV) * (cb - cfb)[..., None]

    _check(w, image, 1024, 2e-2)


def test_emission_seam_and_flat_fold():
    """A square whose two triangles emit differently (its diagonal is a seam), beside a
    strip folded along its middle with one emission (a crease without a jump)."""
    EA, EB = np.array([0.8, 0.5, 0.3]), np.array([0.3, 0.7, 0.2])
    seam = synth.quad_mesh(SQUARE)
    seam.emission = np.stack([EA, EB]).astype(F32)
    fold_pts = [(-1.0, -0.5, 0.0), (-0.75, -0.5, 0.2), (-0.5, -0.5, 0.0), (-0.5, 0.45, 0.0),
                (-0.75, 0.45, 0.2), (-1.0, 0.45, 0.0)]
    fold = synth.Mesh(np.asarray(fold_pts, F32), np.array([[0, 1, 4], [0, 4, 5], [1, 2, 3], [1, 3, 4]], np.int32),
                      np.zeros((4, 3, 2), F32))
    EF = np.array([0.5, 0.4, 0.6])
    fold.emission = np.tile(EF.astype(F32), (4, 1))
    w = _workload(synth._merge([seam, fold]), _cam(eye=(0.1, 0.05, 2.2)))
    tri = [[SQUARE[0], SQUARE[1], SQUARE[2]], [SQUARE[0], SQUARE[2], SQUARE[3]]]
    halves = [[fold_pts[0], fold_pts[1], fold_pts[4], fold_pts[5]], [fold_pts[1], fold_pts[2], fold_pts[3], fold_pts[4]]]

    def image(K, R, t):
        img = np.tile(ENV, (24, 24, 1))
        for pts, e in zip(tri, (EA, EB)):
            img += (e - ENV) * pixel_areas(image_polygon(K, R, t, pts), 24, 24)[..., None]
        for pts in halves:   # the two halves of the fold do not overlap in this view
            img += (EF - ENV) * pixel_areas(image_polygon(K, R, t, pts), 24, 24)[..., None]
        return img

    # the fold lies beside the square's image, and its halves do not overlap each other
    K, R, t = w.camera.K, w.camera.R, w.camera.t
    sq = image_polygon(K, R, t, SQUARE)
    hp = [image_polygon(K, R, t, pts) for pts in halves]
    assert all(area(clip_convex(h, sq)) == 0.0 for h in hp) and area(clip_convex(hp[0], hp[1])) < 1e-9
    _check(w, image, 1024, 2e-2)


def test_closed_box():
    """A closed box, each face emitting its own colour: the visible faces tile its image
    (convex solid), the hidden ones add nothing."""
    lo, hi = np.array([-0.3, -0.25, 0.0]), np.array([0.25, 0.3, 0.45])
    box = synth.box_mesh(lo, hi)
    rng = np.random.default_rng(7)
    face_e = rng.uniform(0.2, 1.0, (6, 3))
    box.emission = np.repeat(face_e, 2, axis=0).astype(F32)
    cam = _cam(eye=(0.9, 0.7, 1.6), target=(0.0, 0.0, 0.2), fov=45.0)
    w = _workload(box, cam)
    V, T = box.vertices.astype(np.float64), box.triangles
    faces = [[V[T[2 * f, 0]], V[T[2 * f, 1]], V[T[2 * f, 2]], V[T[2 * f + 1, 2]]] for f in range(6)]
    centre = 0.5 * (lo + hi)

    def image(K, R, t):
        o = -R.T @ t
        img = np.tile(ENV, (24, 24, 1))
        for f, pts in enumerate(faces):
            c = np.mean(pts, axis=0)
            n = c - centre   # outward for an axis-aligned box face
            if np.dot(n, o - c) > 0:
                img += (face_e[f] - ENV) * pixel_areas(image_polygon(K, R, t, pts), 24, 24)[..., None]
        return img

    # the faces as quads: every quad of box_mesh is triangles (0, 1, 2), (0, 2, 3)
    for f in range(6):
        assert (T[2 * f + 1] == [T[2 * f, 0], T[2 * f, 2], T[2 * f + 1, 2]]).all()
    _check(w, image, 1024, 2e-2)


def test_box_of_one_emission_without_seams():
    """The same box with one emission and no texture seams: only its silhouette, where a
    visible face meets a hidden one at an angle, has a jump."""
    lo, hi = np.array([-0.3, -0.25, 0.0]), np.array([0.25, 0.3, 0.45])
    box = synth.box_mesh(lo, hi)
    box.corner_uvs[:] = 0.0
    EB = np.array([0.7, 0.45, 0.25])
    box.emission = np.tile(EB.astype(F32), (12, 1))
    w = _workload(box, _cam(eye=(0.9, 0.7, 1.6), target=(0.0, 0.0, 0.2), fov=45.0))
    V, T = box.vertices.astype(np.float64), box.triangles
    faces = [[V[T[2 * f, 0]], V[T[2 * f, 1]], V[T[2 * f, 2]], V[T[2 * f + 1, 2]]] for f in range(6)]
    centre = 0.5 * (lo + hi)

    def image(K, R, t):
        o = -R.T @ t
        cov = np.zeros((24, 24))
        for pts in faces:
            c = np.mean(pts, axis=0)
            if np.dot(c - centre, o - c) > 0:
                cov += pixel_areas(image_polygon(K, R, t, pts), 24, 24)
        return ENV + (EB - ENV) * cov[..., None]

    _check(w, image, 1024, 2e-2)


def test_faces_folded_flat():
    """Two coplanar triangles of one emission on the same side of their common edge (folded
    flat): the edge bounds what they cover together."""
    A, B = (-0.3, -0.3, 0.3), (0.3, -0.25, 0.3)
    C0, C1 = (0.0, 0.35, 0.3), (0.15, 0.1, 0.3)
    m = synth.Mesh(np.asarray([A, B, C0, C1], F32), np.array([[0, 1, 2], [0, 1, 3]], np.int32),
                   np.zeros((2, 3, 2), F32))
    m.emission = np.tile(E1.astype(F32), (2, 1))
    w = _workload(m, _cam())

    def image(K, R, t):
        t0, t1 = image_polygon(K, R, t, [A, B, C0]), image_polygon(K, R, t, [A, B, C1])
        cov = pixel_areas(t0, 24, 24) + pixel_areas(t1, 24, 24) - pixel_areas(clip_convex(t1, t0), 24, 24)
        return ENV + (E1 - ENV) * cov[..., None]

    _check(w, image, 1024, 2e-2)


def _with_degenerate_faces(m):
    """m plus a sliver glued to its first edge (third corner on that edge, its own vertex)
    and a triangle with a repeated corner: neither covers any area."""
    A, B = m.vertices[0], m.vertices[1]
    V = np.concatenate([m.vertices, ((A + B) / 2)[None]]).astype(F32)
    nv = m.vertices.shape[0]
    T = np.concatenate([m.triangles, [[0, 1, nv], [1, 1, 2]]]).astype(np.int32)
    UV = np.concatenate([m.corner_uvs, np.zeros((2, 3, 2), F32)]).astype(F32)
    out = synth.Mesh(V, T, UV)
    if m.emission is not None:
        out.emission = np.concatenate([m.emission, np.repeat(m.emission[:1], 2, axis=0)]).astype(F32)
    return out


def test_faces_of_no_area_take_no_part():
    """A sliver glued to the square's edge and a triangle with a repeated corner change
    nothing: they are never seen, and the edge they share stays one silhouette."""
    w = _workload(_with_degenerate_faces(_emissive(SQUARE, E1)), _cam())
    _check(w, _square_image, 1024, 2e-2)


def test_floor_reaching_behind_the_camera():
    """A large emissive floor seen at a grazing angle from just above it: its near edges
    pass behind the camera and are clipped at the camera plane; only the far edge and the
    side edges' visible parts are in the image."""
    EF = np.array([0.6, 0.3, 0.5])
    floor = _emissive([(-1.5, -3.0, 0.0), (1.2, -3.0, 0.0), (1.3, 1.5, 0.0), (-1.4, 1.4, 0.0)], EF)
    cam = synth.pinhole((0.1, -1.0, 0.25), (0.0, 1.0, 0.1), 60.0, 24, 24, up=(0, 0, 1))
    w = _workload(floor, cam)
    pts = [(-1.5, -3.0, 0.0), (1.2, -3.0, 0.0), (1.3, 1.5, 0.0), (-1.4, 1.4, 0.0)]

    def image(K, R, t):
        return ENV + (EF - ENV) * pixel_areas(image_polygon(K, R, t, pts, wmin=1e-3), 24, 24)[..., None]

    _check(w, image, 1024, 2e-2)


def test_lambert_square_under_the_environment():
    """A Lambert square of albedo rho, lit by the environment only, nothing above it: every
    sample on it is rho * L_env (depth 1 and 2: the bounce escapes and a path sees the
    environment directly only from the camera)."""
    rho = 0.6
    m = synth.quad_mesh(SQUARE)
    for depth in (1, 2):
        w = _workload(m, _cam(), albedo=rho, max_depth=depth)

        def image(K, R, t):
            cov = pixel_areas(image_polygon(K, R, t, SQUARE), 24, 24)
            return ENV + (rho * ENV - ENV) * cov[..., None]

        _check(w, image, 1024, 2e-2)


def test_texture_seam_under_the_environment():
    """A Lambert square whose two triangles read different albedo texels (all corners of
    one triangle at one texture coordinate, of the other at another): its diagonal is a
    texture seam with the jump (rho0 - rho1) L_env."""
    rho0, rho1 = 0.7, 0.25
    m = synth.quad_mesh(SQUARE)
    m.corner_uvs[0] = (0.1, 0.5)
    m.corner_uvs[1] = (0.9, 0.5)
    w = _workload(m, _cam())
    w.albedo[:, :2] = rho0
    w.albedo[:, 2:] = rho1
    tri = [[SQUARE[0], SQUARE[1], SQUARE[2]], [SQUARE[0], SQUARE[2], SQUARE[3]]]

    def image(K, R, t):
        img = np.tile(ENV, (24, 24, 1))
        for pts, rho in zip(tri, (rho0, rho1)):
            img += (rho * ENV - ENV) * pixel_areas(image_polygon(K, R, t, pts), 24, 24)[..., None]
        return img

    _check(w, image, 1024, 2e-2)


def test_full_vjp_adds_the_boundary_part():
    """render_vjp with edge_density adds the boundary part to the interior one: on the
    emissive square the interior part is zero, and the total matches the exact gradient."""
    w = _workload(_emissive(SQUARE, E1), _cam())
    G = np.random.default_rng(2).normal(size=(24, 24, 3))
    exact = _exact_gradient(_square_image, w.camera, G)
    g0 = O.render_vjp(O.Scene(w), G, camera=True)
    assert np.abs(np.concatenate([g0["camera_R"].ravel(), g0["camera_t"]])).max() < 1e-9
    g = O.render_vjp(O.Scene(w, edge_density=1024), G, camera=True)
    tot = np.concatenate([g["camera_R"].ravel(), g["camera_t"]])
    np.testing.assert_allclose(tot, exact, rtol=0, atol=2e-2 * np.abs(exact).max())
