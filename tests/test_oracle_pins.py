"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a published value, a closed form derived by a
different route than the oracle's own formula, a library routine, an invariant,
brute force, or finite differences.  A dropped term, a wrong sign or index, or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, ndimage, spatial, stats

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="session", autouse=True)
def _built():
    O.build(force=False)


# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al. SC'11)
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        got = O.philox(key[0] | (key[1] << 32), np.array([ctr], np.uint32))[0]
        assert [int(x) for x in got] == want


def test_philox_uniformity_chi2():
    n = 1 << 17
    c = np.zeros((n, 4), np.uint32)
    c[:, 0] = np.arange(n) % 4096
    c[:, 1] = np.arange(n) // 4096
    c[:, 2] = 3
    x = O.philox(12345, c)
    u = (x >> 8).astype(np.float64) * 2.0 ** -24
    assert u.min() >= 0.0 and u.max() < 1.0
    for k in range(4):
        h, _ = np.histogram(u[:, k], bins=256, range=(0, 1))
        assert stats.chisquare(h).pvalue > 1e-4
    # neighbouring counters are uncorrelated
    r = np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]
    assert abs(r) < 0.02


# ---------------------------------------------------------------------------
# camera rays (Eq. 6 inverted): the first hit projects back to the jittered pixel
# ---------------------------------------------------------------------------

def test_camera_ray_round_trip():
    w = synth.quad_cube()
    sc = O.Scene(w)
    rng = np.random.default_rng(0)
    for _ in range(200):
        pix = int(rng.integers(0, 64 * 64))
        s = int(rng.integers(0, 4))
        h = O.first_hit(sc, pix, s)
        assert h["prim"] >= 0
        uv, _ = scenes.project(w.camera.K, w.camera.R, w.camera.t, h["x"][None])
        u = scenes.philox_u(w.seed, pix, s, 0)
        want = np.array([pix % 64 + u[0], pix // 64 + u[1]])
        np.testing.assert_allclose(uv[0], want, rtol=0, atol=1e-9)
        # the ray starts at the camera centre
        np.testing.assert_allclose(h["o"], -w.camera.R.T @ w.camera.t, atol=1e-12)


# ---------------------------------------------------------------------------
# projector next-event estimation (Eq. 1-3, 6)
# ---------------------------------------------------------------------------

def _direct_check(w, expect_fn, skip_fn=lambda h: False, atol=1e-12):
    sc = O.Scene(w)
    out = O.render(sc)
    L = out["L"]
    W = w.camera.width
    n_checked = 0
    for pix in range(w.camera.width * w.camera.height):
        for s in range(w.spp):
            h = O.first_hit(sc, pix, s)
            if h["prim"] < 0 or skip_fn(h):
                continue
            exp = expect_fn(h)
            np.testing.assert_allclose(L[pix, s], exp, rtol=1e-11, atol=atol,
                                       err_msg=f"pixel {pix % W},{pix // W} sample {s}")
            n_checked += 1
    return n_checked


def _in_frustum_margin(w, x):
    uv, p = scenes.project(w.projector.K, w.projector.R, w.projector.t, x[None])
    u, v = uv[0]
    m = min(u, w.projector.width - u, v, w.projector.height - v)
    return m, p[0, 2]


def test_fronto_parallel_plane_irradiance():
    """Projector axis normal to the plane: irradiance is E_p / z0^2 everywhere in the frustum."""
    w = scenes.plane_workload(proj_eye=(0.0, 0.0, 1.0))
    Ep = w.prf_gain * float(np.float32(0.6)) ** 2.2
    rho = 0.5

    def expect(h):
        m, z = _in_frustum_margin(w, h["x"])
        return np.full(3, rho / math.pi * Ep / z ** 2) if m > 0 else np.zeros(3)

    n = _direct_check(w, expect, skip_fn=lambda h: abs(_in_frustum_margin(w, h["x"])[0]) < 1e-6)
    assert n > 3000


def test_tilted_plane_irradiance_by_flux_conservation():
    """Irradiance on a tilted plane = E_p * |d(u,v)/d(x,y)| / (f_x f_y) (flux of each
    image-plane element lands on its footprint), independent of the cos/d^2 form."""
    a = scenes.deg(35.0)
    w = scenes.plane_workload(proj_eye=(-0.8 * math.sin(a), 0.1, 0.8 * math.cos(a)))
    Ep = w.prf_gain * float(np.float32(0.6)) ** 2.2
    rho = 0.5
    K, R, t = w.projector.K, w.projector.R, w.projector.t
    fxfy = K[0, 0] * K[1, 1]

    def jac(x):
        e = 1e-6
        def uv(px, py):
            return scenes.project(K, R, t, np.array([[px, py, 0.0]]))[0][0]
        du = (uv(x[0] + e, x[1]) - uv(x[0] - e, x[1])) / (2 * e)
        dv = (uv(x[0], x[1] + e) - uv(x[0], x[1] - e)) / (2 * e)
        return abs(du[0] * dv[1] - du[1] * dv[0])

    def expect(h):
        m, _ = _in_frustum_margin(w, h["x"])
        return np.full(3, rho / math.pi * Ep * jac(h["x"]) / fxfy) if m > 0 else np.zeros(3)

    sc = O.Scene(w)
    L = O.render(sc)["L"]
    checked = 0
    for pix in range(0, 32 * 32, 3):
        for s in range(w.spp):
            h = O.first_hit(sc, pix, s)
            if h["prim"] < 0 or abs(_in_frustum_margin(w, h["x"])[0]) < 1e-6:
                continue
            # central differences of the projection: relative accuracy ~1e-8
            np.testing.assert_allclose(L[pix, s], expect(h), rtol=1e-6, atol=1e-12)
            checked += 1
    assert checked > 800


def test_texture_lookup_against_library_bilinear():
    """Albedo fetched bilinearly at the affine UV of the hit point (scipy map_coordinates)."""
    rng = np.random.default_rng(4)
    tex = rng.uniform(0.1, 0.9, (16, 16, 3)).astype(np.float32)
    w = scenes.plane_workload(proj_eye=(0.0, 0.0, 1.0), tex=tex, half=0.3, cam_eye=(0.0, 0.05, 0.5),
                              proj_fov=80.0)
    Ep = w.prf_gain * float(np.float32(0.6)) ** 2.2

    def expect(h):
        m, z = _in_frustum_margin(w, h["x"])
        if m <= 0:
            return np.zeros(3)
        hf = float(np.float32(0.3))   # the quad's corners are stored as float32
        u = (h["x"][0] + hf) / (2 * hf)
        v = (h["x"][1] + hf) / (2 * hf)
        a = [ndimage.map_coordinates(tex[..., c].astype(np.float64), [[v * 16 - 0.5], [u * 16 - 0.5]],
                                     order=1, mode="nearest")[0] for c in range(3)]
        return np.array(a) / math.pi * Ep / z ** 2

    n = _direct_check(w, expect, skip_fn=lambda h: abs(_in_frustum_margin(w, h["x"])[0]) < 1e-6)
    assert n > 3000


def test_projector_image_bilinear_against_library():
    rng = np.random.default_rng(9)
    img = rng.uniform(0, 1, (7, 9, 3))
    xy = rng.uniform(-2, 11, (500, 2))
    got = O.bilinear(img, xy)
    want = np.stack([ndimage.map_coordinates(img[..., c], [xy[:, 1], xy[:, 0]], order=1, mode="nearest")
                     for c in range(3)], 1)
    np.testing.assert_allclose(got, want, atol=1e-14)


def test_hard_shadow_of_the_cube():
    """Quad-and-cube geometry, direct only: samples on the floor inside the cube's shadow polygon
    (convex hull of the cube's corners projected from the projector centre) receive nothing;
    the others follow the flux-conservation closed form."""
    w = scenes.c1_direct()
    K, R, t = w.projector.K, w.projector.R, w.projector.t
    op = -R.T @ t
    cube = np.array([[x, y, z] for x in (0.05, 0.25) for y in (-0.1, 0.1) for z in (0.0, 0.2)])
    shadow = np.array([op + (c - op) * (op[2] / (op[2] - c[2])) for c in cube])[:, :2]
    hull = spatial.Delaunay(shadow)
    hull_pts = shadow[spatial.ConvexHull(shadow).vertices]
    Ep = 1.0 * float(np.float32(0.8)) ** 2.2
    fxfy = K[0, 0] * K[1, 1]

    def seg_dist(p, a, b):
        ab = b - a
        s = np.clip(np.dot(p - a, ab) / np.dot(ab, ab), 0, 1)
        return np.linalg.norm(p - (a + s * ab))

    def border(p):
        return min(seg_dist(p, hull_pts[i], hull_pts[(i + 1) % len(hull_pts)]) for i in range(len(hull_pts)))

    def jac(x):
        e = 1e-6
        uv = lambda px, py: scenes.project(K, R, t, np.array([[px, py, 0.0]]))[0][0]
        du = (uv(x[0] + e, x[1]) - uv(x[0] - e, x[1])) / (2 * e)
        dv = (uv(x[0], x[1] + e) - uv(x[0], x[1] - e)) / (2 * e)
        return abs(du[0] * dv[1] - du[1] * dv[0])

    sc = O.Scene(w)
    L = O.render(sc)["L"]
    n_shadow = n_lit = 0
    for pix in range(64 * 64):
        for s in range(w.spp):
            h = O.first_hit(sc, pix, s)
            if h["prim"] not in (0, 1):
                continue
            x = h["x"]
            m, _ = _in_frustum_margin(w, x)
            if abs(m) < 1e-6 or border(x[:2]) < 1e-6:
                continue
            if m > 0 and hull.find_simplex(x[:2]) >= 0:
                np.testing.assert_array_equal(L[pix, s], 0.0)
                n_shadow += 1
            else:
                exp = 0.6 / math.pi * Ep * jac(x) / fxfy if m > 0 else 0.0
                np.testing.assert_allclose(L[pix, s], exp, rtol=1e-6, atol=1e-12)
                n_lit += 1
    assert n_shadow > 100 and n_lit > 5000


# ---------------------------------------------------------------------------
# interreflection: white furnace (closed Lambertian box, emission Le everywhere)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("depth", [1, 2, 5])
def test_white_furnace_geometric_series(depth):
    rho = 0.7
    w = scenes.furnace_workload(rho=rho, max_depth=depth)
    out = O.render(O.Scene(w))
    rho = float(np.float32(rho))   # textures are float32
    want = sum(rho ** k for k in range(depth))
    np.testing.assert_allclose(out["L"], want, rtol=1e-12)
    np.testing.assert_allclose(out["Ec"], want, rtol=1e-12)


def test_convex_scene_is_depth_invariant():
    w1 = scenes.plane_workload(max_depth=1)
    w4 = scenes.plane_workload(max_depth=4)
    a = O.render(O.Scene(w1))["L"]
    b = O.render(O.Scene(w4))["L"]
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------------------
# linearity of light transport in the projector image
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ggx", [False, True])
def test_linearity_in_projector_image(ggx):
    w = scenes.linear_params(scenes.c3_ggx(spp=2) if ggx else synth.quad_cube(spp=2))
    rng = np.random.default_rng(1)
    I1 = rng.uniform(0, 1, w.proj_image.shape)
    I2 = rng.uniform(0, 1, w.proj_image.shape)
    a, b = 0.3, 1.7
    L1 = O.render(O.Scene(w, proj_image=I1))["L"]
    L2 = O.render(O.Scene(w, proj_image=I2))["L"]
    L12 = O.render(O.Scene(w, proj_image=a * I1 + b * I2))["L"]
    np.testing.assert_allclose(L12, a * L1 + b * L2, rtol=1e-11, atol=1e-14)
    assert np.abs(L12).max() > 0


# ---------------------------------------------------------------------------
# radiance clipping (Eq. 12), PRF (Eq. 1), CRF (Eq. 5)
# ---------------------------------------------------------------------------

def test_clip_forces_bright_samples_to_threshold():
    w = scenes.plane_workload(proj_eye=(0.0, 0.0, 0.4), cam_eye=(0.0, 0.0, 0.3), half=0.05, cam_fov=10.0)
    w.clip = True
    w.clip_k = 1e-3
    w.white_balance = np.array([0.9, 0.5, 1.3])
    out = O.render(O.Scene(w))
    thr = 1e-3 / 0.5
    assert (out["L"] > thr).all()
    np.testing.assert_allclose(out["Ec"], thr, rtol=1e-15)
    w.clip = False
    out2 = O.render(O.Scene(w))
    np.testing.assert_allclose(out2["Ec"], out["L"].mean(1), rtol=1e-15)


def test_prf_special_cases():
    w = synth.quad_cube()
    rng = np.random.default_rng(2)
    I = rng.uniform(0, 1, w.proj_image.shape)
    sc = O.Scene(w, proj_image=I, prf_gamma=np.ones(3), prf_gain=1.0, prf_mix=np.eye(3))
    np.testing.assert_array_equal(O.prf(sc), I)
    sc = O.Scene(w, proj_image=I, prf_gamma=np.full(3, 2.0), prf_gain=1.0, prf_mix=np.eye(3))
    np.testing.assert_allclose(O.prf(sc), I * I, rtol=1e-15)
    perm = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)
    sc = O.Scene(w, proj_image=I, prf_gamma=np.ones(3), prf_gain=2.0, prf_mix=perm)
    np.testing.assert_allclose(O.prf(sc), 2.0 * I[..., [1, 2, 0]], rtol=1e-15)
    sc = O.Scene(w, proj_image=I, prf_gamma=np.ones(3), prf_gain=1.0, prf_mix=-np.eye(3))
    np.testing.assert_array_equal(O.prf(sc), 0.0)


def test_crf_special_cases():
    w = synth.quad_cube()
    w.clip = False   # the clip threshold k / min(w) would differ between the two renders
    a = O.render(O.Scene(w, crf_gamma=np.ones(3), crf_gain=1.0, white_balance=np.ones(3)))
    np.testing.assert_array_equal(a["Ic"], a["Ec"])
    b = O.render(O.Scene(w, crf_gamma=np.full(3, 0.5), crf_gain=4.0, white_balance=np.array([1.0, 0.25, 2.0])))
    np.testing.assert_allclose(b["Ic"] ** 2, a["Ec"] * np.array([4.0, 1.0, 8.0]), rtol=1e-13)


# ---------------------------------------------------------------------------
# BRDF
# ---------------------------------------------------------------------------

def _rand_dir(rng, n):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    return v if v @ n > 0 else -v


def test_brdf_helmholtz_reciprocity():
    rng = np.random.default_rng(3)
    for _ in range(300):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        a, b = _rand_dir(rng, n), _rand_dir(rng, n)
        alb = rng.uniform(0, 1, 3)
        r, sp = rng.uniform(0.05, 1), rng.uniform(0, 1)
        for kind in (0, 1):
            f1 = O.brdf(kind, n, a, b, alb, r, sp)
            f2 = O.brdf(kind, n, b, a, alb, r, sp)
            np.testing.assert_allclose(f1, f2, rtol=1e-12, atol=1e-15)


def test_brdf_lambert_and_normal_incidence_peak():
    n = np.array([0.0, 0.0, 1.0])
    alb = np.array([0.2, 0.5, 0.9])
    wi = np.array([0.3, -0.2, 0.9]) / np.linalg.norm([0.3, -0.2, 0.9])
    wo = np.array([-0.5, 0.1, 0.6]) / np.linalg.norm([-0.5, 0.1, 0.6])
    np.testing.assert_allclose(O.brdf(0, n, wo, wi, alb, 0.3, 0.7)[:3], alb / math.pi, rtol=1e-15)
    # GGX at wi = wo = n: D = 1/(pi a^2), G = 1, F = F0 = 0.08 sp
    for r, sp in [(0.3, 0.7), (0.8, 0.0), (0.5, 1.0)]:
        a = r * r
        want = alb / math.pi + 0.08 * sp / (math.pi * a * a) / 4.0
        np.testing.assert_allclose(O.brdf(1, n, n, n, alb, r, sp)[:3], want, rtol=1e-13)
    # below the horizon: zero
    assert np.all(O.brdf(1, n, wo, -wi, alb, 0.3, 0.7)[:3] == 0)


@pytest.mark.parametrize("r", [0.1, 0.35, 0.6, 0.95])
def test_ggx_ndf_projected_area_is_one(r):
    val, err = integrate.quad(lambda mu: 2 * math.pi * O.ggx_D(mu, r) * mu, 0.0, 1.0, limit=400,
                              points=[0.99, 0.999, 0.9999])
    assert abs(val - 1.0) < 1e-6


def test_ggx_smith_g1_matches_lambda_form():
    for r in (0.1, 0.4, 0.8):
        a = r * r
        for c in np.linspace(0.05, 1.0, 20):
            tan2 = (1 - c * c) / (c * c)
            lam = (-1 + math.sqrt(1 + a * a * tan2)) / 2
            assert abs(O.ggx_G1(c, r) - 1.0 / (1.0 + lam)) < 1e-13


def test_brdf_derivatives_match_finite_differences():
    rng = np.random.default_rng(8)
    for _ in range(100):
        n = np.array([0.0, 0.0, 1.0])
        wo, wi = _rand_dir(rng, n), _rand_dir(rng, n)
        alb = rng.uniform(0, 1, 3)
        r, sp = rng.uniform(0.1, 1), rng.uniform(0, 1)
        g = O.brdf(1, n, wo, wi, alb, r, sp)
        h = 1e-6
        fr = (O.brdf(1, n, wo, wi, alb, r + h, sp)[0] - O.brdf(1, n, wo, wi, alb, r - h, sp)[0]) / (2 * h)
        fs = (O.brdf(1, n, wo, wi, alb, r, sp + h)[0] - O.brdf(1, n, wo, wi, alb, r, sp - h)[0]) / (2 * h)
        assert abs(fr - g[3]) <= 1e-6 * max(1.0, abs(g[3]))
        assert abs(fs - g[4]) <= 1e-7 * max(1.0, abs(g[4]))


def _sphere_grid(nt, nphi):
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    dw = (np.sin(T) * (math.pi / nt) * (2 * math.pi / nphi)).reshape(-1)
    return d, dw


@pytest.mark.parametrize("kind,r", [(0, 0.5), (1, 0.5), (1, 0.9), (1, 0.7)])
def test_bounce_pdf_integrates_to_one(kind, r):
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.4, 0.1, 0.8]) / np.linalg.norm([0.4, 0.1, 0.8])
    d, dw = _sphere_grid(1500, 3000)
    p = O.pdf_batch(kind, n, wo, r, d)
    assert abs((p * dw).sum() - 1.0) < 2e-3


@pytest.mark.parametrize("kind,r", [(0, 0.5), (1, 0.3), (1, 0.8)])
def test_bounce_sampler_matches_its_pdf(kind, r):
    """Histogram of sampled directions (chi-square) against the pdf integrated per bin."""
    rng = np.random.default_rng(21)
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.5, -0.2, 0.7]) / np.linalg.norm([0.5, -0.2, 0.7])
    N = 200000
    wi, _ = O.sample(kind, n, wo, r, rng.uniform(0, 1, (N, 3)))
    nt, nph = 12, 16
    th = np.arccos(np.clip(wi[:, 2], -1, 1))
    ph = np.mod(np.arctan2(wi[:, 1], wi[:, 0]), 2 * math.pi)
    obs, _, _ = np.histogram2d(th, ph, bins=[nt, nph], range=[[0, math.pi], [0, 2 * math.pi]])
    d, dw = _sphere_grid(nt * 60, nph * 60)
    p = O.pdf_batch(kind, n, wo, r, d) * dw
    exp = p.reshape(nt, 60, nph, 60).sum(axis=(1, 3)) * N
    mask = exp > 20
    chi = ((obs[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    assert stats.chi2.sf(chi, mask.sum() - 1) > 1e-4
    assert obs[~mask].sum() <= max(40, 3 * exp[~mask].sum())


# ---------------------------------------------------------------------------
# ray / triangle
# ---------------------------------------------------------------------------

def _tri_scene(V, F):
    mesh = synth.Mesh(np.asarray(V, np.float32), np.asarray(F, np.int32),
                      np.zeros((len(F), 3, 2), np.float32))
    w = synth.quad_cube()
    w.mesh = mesh
    return O.Scene(w, tmin=1e-6)


def test_triangle_hits_by_hand():
    sc = _tri_scene([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, -1], [1, 0, -1], [0, 1, -1]],
                    [[0, 1, 2], [3, 4, 5], [0, 1, 2]])
    rays = np.array([
        [0.2, 0.3, 1.0, 0, 0, -1, 1e300, -1],   # hits prims 0 and 2 at t=1 -> tie -> 0
        [0.2, 0.3, 1.0, 0, 0, -1, 1e300, 0],    # skip 0 -> 2
        [0.2, 0.3, 1.0, 0, 0, -1, 1.0, -1],     # t must be < tmax (exclusive) -> miss
        [0.7, 0.7, 1.0, 0, 0, -1, 1e300, -1],   # outside (b0 < 0) -> miss
        [0.5, 0.5, 1.0, 0, 0, -1, 1e300, -1],   # on the hypotenuse: b0 = 0, inclusive
        [0.2, 0.3, -2.0, 0, 0, 1, 1e300, -1],   # from below: nearest is the lower triangle (prim 1)
        [0.2, 0.3, 1.0, 1, 0, 0, 1e300, -1],    # parallel to the plane -> miss
    ])
    prim, t, b1, b2 = O.intersect(sc, rays)
    assert list(prim) == [0, 2, -1, -1, 0, 1, -1]
    assert t[0] == 1.0 and abs(b1[0] - 0.2) < 1e-15 and abs(b2[0] - 0.3) < 1e-15
    assert t[5] == 1.0


def test_margin_flags_near_edge_rays():
    sc = _tri_scene([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], [[0, 1, 2], [1, 3, 2]])
    diag = math.sqrt(2)
    tx = 2e-6 * diag
    eps = [0.1 * tx, 10 * tx]
    rays = []
    for e in eps:   # close to / away from the shared edge x + y = 1
        rays.append([0.5 - e, 0.5 - e, 1, 0, 0, -1, 1e300, -1])
    prim, t, _, _, m = O.intersect(sc, np.array(rays), with_margin=True)
    assert list(prim) == [0, 0]
    assert m[0] < 1 and m[1] > 1


def test_clean_samples_survive_fp32_level_perturbation():
    """The margin protocol: shifting the camera and projector poses by float32-rounding
    amounts (1e-7 relative) changes no hit on samples the unperturbed oracle marks clean."""
    w = synth.corner_50k(spp=2, n_quads=16, res=24)
    base = O.render(O.Scene(w), want=("hits", "margin"))
    rng = np.random.default_rng(5)
    cam, prj = w.camera, w.projector
    jig = lambda a: np.asarray(a) * (1 + rng.uniform(-1, 1, np.shape(a)) * 1.2e-7)
    cam2 = synth.Pinhole(jig(cam.K), cam.R, jig(cam.t), cam.width, cam.height)
    prj2 = synth.Pinhole(jig(prj.K), prj.R, jig(prj.t), prj.width, prj.height)
    pert = O.render(O.Scene(w, camera=cam2, projector=prj2), want=("hits",))
    clean = base["margin"] >= 1
    assert clean.mean() > 0.97
    np.testing.assert_array_equal(pert["hits"][clean], base["hits"][clean])


# ---------------------------------------------------------------------------
# adjoint: dot-product test and finite differences of the frozen-path estimator
# ---------------------------------------------------------------------------

def test_adjoint_dot_product_on_linear_map():
    """With gamma = 1, unit gains and no clipping the render is a linear map A of I_p;
    the VJP must satisfy <G, A v> = <A^T G, v>."""
    w = scenes.linear_params(scenes.c3_ggx(spp=2))
    rng = np.random.default_rng(13)
    v = rng.uniform(0, 1, w.proj_image.shape)
    G = rng.normal(size=(64, 64, 3))
    Av = O.render(O.Scene(w, proj_image=v))["Ic"].reshape(64, 64, 3)
    g = O.render_vjp(O.Scene(w, proj_image=v), G)
    lhs = (G * Av).sum()
    rhs = (g["Ip"] * v).sum()
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def _fd_params(w, rng, count):
    """Random differentiable parameters of a workload: (group, index) pairs."""
    choices = []
    th, tw = w.albedo.shape[:2]
    for _ in range(count):
        g = rng.choice(["Ip", "albedo", "roughness", "specular", "prf_gamma", "prf_mix", "crf_gamma",
                        "white_balance"], p=[0.3, 0.2, 0.15, 0.15, 0.05, 0.05, 0.05, 0.05])
        if g == "Ip":
            idx = (int(rng.integers(16, 48)), int(rng.integers(16, 48)), int(rng.integers(0, 3)))
        elif g == "albedo":
            idx = (int(rng.integers(0, th)), int(rng.integers(0, tw)), int(rng.integers(0, 3)))
        elif g in ("roughness", "specular"):
            idx = (int(rng.integers(0, th)), int(rng.integers(0, tw)))
        elif g == "prf_mix":
            idx = (int(rng.integers(0, 3)), int(rng.integers(0, 3)))
        else:
            idx = (int(rng.integers(0, 3)),)
        choices.append((g, idx))
    return choices


def _loss(w, G, overrides):
    return float((O.render(O.Scene(w, **overrides), want=("Ic",))["Ic"].reshape(G.shape) * G).sum())


@pytest.mark.parametrize("clip,env", [(False, 0.0), (True, 0.0), (False, 0.4)])
def test_adjoint_matches_central_differences(clip, env):
    """64 random parameters, central differences h = 1e-3 of the frozen-path estimator
    (directions sampled with the unperturbed roughness); with env > 0 every vertex also
    samples the environment (GGX lobes, occlusion by the cube), so the adjoint of that
    next-event term is checked as well."""
    w = scenes.c3_ggx(spp=3, seed=17)
    w.clip = clip
    w.clip_k = 0.35 if clip else 1.0
    w.env = np.array([1.0, 0.8, 0.6]) * env
    rng = np.random.default_rng(302)
    G = rng.normal(size=(64, 64, 3))
    base = dict(proj_image=w.proj_image.astype(np.float64), albedo=w.albedo.astype(np.float64),
                roughness=w.roughness.astype(np.float64), specular=w.specular.astype(np.float64),
                prf_gamma=np.array(w.prf_gamma, float), prf_mix=np.array(w.prf_mix, float),
                crf_gamma=np.array(w.crf_gamma, float), white_balance=np.array(w.white_balance, float))
    grad = O.render_vjp(O.Scene(w, rough_sample=base["roughness"], **base), G)
    gmap = dict(proj_image=grad["Ip"], albedo=grad["albedo"], roughness=grad["roughness"],
                specular=grad["specular"], prf_gamma=grad["prf_gamma"], prf_mix=grad["prf_mix"],
                crf_gamma=grad["crf_gamma"], white_balance=grad["white_balance"])
    if clip:   # make sure the clip branch and the threshold gradient are exercised
        L = O.render(O.Scene(w, **base))["L"]
        assert ((L > 0.35 / w.white_balance.min()).mean()) > 0.01
    h = 1e-3
    worst = 0.0
    count = 0
    for g, idx in _fd_params(w, rng, 64):
        key = "proj_image" if g == "Ip" else g
        ad = gmap[key][idx]

        def at(delta):
            o = {k: v.copy() for k, v in base.items()}
            o[key][idx] += delta
            out = O.render(O.Scene(w, rough_sample=base["roughness"], **o), want=("Ic", "L"))
            thr = w.clip_k / o["white_balance"].min()
            return float((out["Ic"].reshape(G.shape) * G).sum()), out["L"] > thr

        (fp, mp), (fm, mm) = at(h), at(-h)
        if clip and not np.array_equal(mp, mm):
            continue   # a sample crosses the clip kink inside [-h, h]: FD is not a derivative there
        fd = (fp - fm) / (2 * h)
        err = abs(fd - ad) / max(abs(ad), abs(fd), 1e-6)
        worst = max(worst, err)
        count += 1
        assert err < 2e-4 or abs(fd - ad) < 1e-7, (g, idx, fd, ad)
    assert count >= (48 if clip else 64)


def test_clip_threshold_gradient_by_finite_differences():
    """d/dw of the channel with the smallest white balance flows through the clip threshold
    k / min(w) (Eq. 12) as well as the CRF; FD step small enough that no sample crosses the kink."""
    w = scenes.c3_ggx(spp=3, seed=17)
    w.clip = True
    w.clip_k = 0.35
    rng = np.random.default_rng(302)
    G = rng.normal(size=(64, 64, 3))
    wb = np.array(w.white_balance, float)
    a = int(np.argmin(wb))
    g = O.render_vjp(O.Scene(w, white_balance=wb), G)["white_balance"]
    h = 1e-5
    vals, masks = [], []
    for dl in (h, -h):
        wb2 = wb.copy()
        wb2[a] += dl
        out = O.render(O.Scene(w, white_balance=wb2), want=("Ic", "L"))
        vals.append((out["Ic"].reshape(G.shape) * G).sum())
        masks.append(out["L"] > w.clip_k / wb2.min())
    assert np.array_equal(masks[0], masks[1]) and masks[0].any()
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(fd - g[a]) <= 1e-7 * abs(g[a])
    # the threshold term is not negligible: removing it changes the gradient
    w.clip = False
    g_noclip = O.render_vjp(O.Scene(w, white_balance=wb), G)["white_balance"]
    assert abs(g_noclip[a] - g[a]) > 1e-3 * abs(g[a])
