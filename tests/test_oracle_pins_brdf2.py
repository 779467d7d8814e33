"""Pins of the oracle's metallic map and normal map (the rest of the principled BRDF's maps
in theta, Sec. 3.2 and 4.3), against closed forms, invariants and finite differences.

Readings (the paper names Burley's principled BRDF and Mitsuba's normal-map convention
without formulas): metallic mu blends the dielectric specular colour 0.08 * specular into
the base colour, F0 = (1 - mu) 0.08 sp + mu a, and scales the diffuse lobe by (1 - mu);
the normal map stores t = 2 v - 1 in the tangent frame T = dP/du (orthogonal to the
geometric normal n), B = n x T, so (0.5, 0.5, 1) leaves the normal unchanged; the BRDF
and the cosine of the rendering equation are taken about the shading normal, and a
direction counts only above both the shading and the geometric surface.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_12174_amd import synth

from . import scenes

F32 = np.float32


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _f32(x):
    return float(np.float32(x))


def _rand_unit(rng, n=None):
    v = rng.normal(size=(3,) if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _upper(rng, n):
    """A random unit direction in the hemisphere of n."""
    while True:
        w = _rand_unit(rng)
        if w @ n > 0.05:
            return w


# ---------------------------------------------------------------------------
# the BRDF with metallic and a shading normal
# ---------------------------------------------------------------------------

def test_metallic_peak_at_normal_incidence():
    """wi = wo = n: h = n, Schlick's factor vanishes (F = F0), D = 1 / (pi a^2), G1 = 1, so
    f_c = (1 - mu) a_c / pi + F0_c / (4 pi a^2), F0_c = (1 - mu) 0.08 sp + mu a_c.  At
    mu = 1 the lobe carries the base colour alone: f_c = a_c / (4 pi a^2)."""
    n = np.array([0.0, 0.0, 1.0])
    a = np.array([0.9, 0.4, 0.1])
    for r, sp, mu in ((0.5, 0.3, 1.0), (0.4, 0.7, 0.0), (0.6, 0.5, 0.35)):
        al = max(r * r, 1e-3)
        b = O.brdf_full(1, n, n, n, n, a, r, sp, mu)
        F0 = (1 - mu) * 0.08 * sp + mu * a
        np.testing.assert_allclose(b["f"], (1 - mu) * a / math.pi + F0 / (4 * math.pi * al * al), rtol=1e-12)
        assert b["c"] == 1.0
    b = O.brdf_full(1, n, n, n, n, a, 0.5, 0.3, 1.0)
    np.testing.assert_allclose(b["f"], a / (4 * math.pi * 0.25 ** 2), rtol=1e-12)


def test_metallic_interpolates_linearly():
    """f is affine in mu (both the diffuse scale and F0 are): f(1/2) = (f(0) + f(1)) / 2,
    and the metallic derivative is f(1) - f(0)."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = _rand_unit(rng)
        wo, wi = _upper(rng, n), _upper(rng, n)
        a = rng.uniform(0.05, 0.95, 3)
        r, sp = rng.uniform(0.1, 0.9), rng.uniform(0, 1)
        f0, f1, fh = (O.brdf_full(1, n, n, wo, wi, a, r, sp, mu) for mu in (0.0, 1.0, 0.5))
        np.testing.assert_allclose(fh["f"], (f0["f"] + f1["f"]) / 2, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(fh["dfm"], f1["f"] - f0["f"], rtol=1e-10, atol=1e-13)


def test_principled_brdf_reciprocity_with_shading_normal():
    """Helmholtz reciprocity f(wo, wi) = f(wi, wo) for directions above both normals."""
    rng = np.random.default_rng(4)
    for _ in range(300):
        ng = _rand_unit(rng)
        ns = ng + 0.3 * _rand_unit(rng)
        ns /= np.linalg.norm(ns)
        while True:
            wo, wi = _rand_unit(rng), _rand_unit(rng)
            if min(wo @ ng, wi @ ng, wo @ ns, wi @ ns) > 0.02:
                break
        a = rng.uniform(0.05, 0.95, 3)
        r, sp, mu = rng.uniform(0.1, 0.9), rng.uniform(0, 1), rng.uniform(0, 1)
        f1 = O.brdf_full(1, ng, ns, wo, wi, a, r, sp, mu)["f"]
        f2 = O.brdf_full(1, ng, ns, wi, wo, a, r, sp, mu)["f"]
        np.testing.assert_allclose(f1, f2, rtol=1e-12)


def test_principled_brdf_derivatives_by_finite_differences():
    """Every derivative the adjoint uses, against central differences of f (and of f times
    the cosine about ns, ns perturbed as a free vector for the normal)."""
    rng = np.random.default_rng(5)
    h = 1e-6
    for kind in (0, 1):
        for _ in range(60):
            ng = _rand_unit(rng)
            ns = ng + 0.2 * _rand_unit(rng)
            ns /= np.linalg.norm(ns)
            while True:
                wo, wi = _rand_unit(rng), _rand_unit(rng)
                if min(wo @ ng, wi @ ng, wo @ ns, wi @ ns) > 0.1:
                    break
            a = rng.uniform(0.1, 0.9, 3)
            r, sp, mu = rng.uniform(0.15, 0.9), rng.uniform(0.05, 0.95), rng.uniform(0.05, 0.95)
            b = O.brdf_full(kind, ng, ns, wo, wi, a, r, sp, mu)
            f = lambda **k: O.brdf_full(kind, k.get("ng", ng), k.get("ns", ns), wo, wi, k.get("a", a), k.get("r", r),
                                        k.get("sp", sp), k.get("mu", mu))
            for c in range(3):
                e = np.zeros(3)
                e[c] = h
                fd = (f(a=a + e)["f"][c] - f(a=a - e)["f"][c]) / (2 * h)
                np.testing.assert_allclose(b["dfa"], fd, rtol=1e-6, atol=1e-9)
            checks = [("dfr", "r", r), ("dfm", "mu", mu)] + ([("dfs", "sp", sp)] if kind else [])
            for key, name, x in checks:
                fd = (f(**{name: x + h})["f"] - f(**{name: x - h})["f"]) / (2 * h)
                np.testing.assert_allclose(np.broadcast_to(b[key], (3,)), fd, rtol=1e-6, atol=1e-9)
            for j in range(3):
                e = np.zeros(3)
                e[j] = h
                p, m = f(ns=ns + e), f(ns=ns - e)
                fd = (p["f"] * p["c"] - m["f"] * m["c"]) / (2 * h)
                np.testing.assert_allclose(b["dfcn"][:, j], fd, rtol=1e-6, atol=1e-9)


def test_directions_below_either_surface_see_nothing():
    """f = 0 when wi is below the shading normal, or below the geometric normal while above
    the shading one (no light through the surface), or when wo is below the shading normal."""
    ng = np.array([0.0, 0.0, 1.0])
    ns = np.array([math.sin(0.5), 0.0, math.cos(0.5)])
    a = np.array([0.5, 0.5, 0.5])
    up = np.array([0.0, 0.0, 1.0])
    grazing_below = np.array([math.cos(0.1), 0.0, -math.sin(0.1)])   # above ns, below ng
    assert grazing_below @ ns > 0 and grazing_below @ ng < 0
    behind = np.array([-math.cos(0.2), 0.0, math.sin(0.2)])          # above ng, below ns
    assert behind @ ng > 0 and behind @ ns < 0
    for kind in (0, 1):
        assert np.all(O.brdf_full(kind, ng, ns, up, grazing_below, a, 0.4, 0.5, 0.3)["f"] == 0)
        assert np.all(O.brdf_full(kind, ng, ns, up, behind, a, 0.4, 0.5, 0.3)["f"] == 0)
        assert np.all(O.brdf_full(kind, ng, ns, behind, up, a, 0.4, 0.5, 0.3)["f"] == 0)
        assert np.all(O.brdf_full(kind, ng, ns, up, up, a, 0.4, 0.5, 0.3)["f"] > 0)


# ---------------------------------------------------------------------------
# the normal map's frame on a textured plane
# ---------------------------------------------------------------------------

def _tilted(theta, phi):
    """stored map value of the tangent-space normal (sin th cos ph, sin th sin ph, cos th)"""
    t = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    return (t + 1) / 2, t


@pytest.mark.parametrize("below", [False, True])
def test_normal_map_tilts_the_shading_normal_on_a_plane(below):
    """A constant normal map on the quad z = 0, whose texture coordinates are u = (x + h)/2h,
    v = (y + h)/2h: dP/du points along +x, so the frame is T = +x, B = n x T and n = +z
    seen from above (B = +y) or -z seen from below (B = -y).  Direct projector light on a
    Lambert plane (fronto-parallel projector, irradiance E_p / z0^2 about n) becomes
    rho / pi * E_p / z0^2 * (ns . wp) / (n . wp) with ns = t_x T + t_y B + t_z n, and 0
    where wp or wo is below ns."""
    theta, phi = math.radians(28.0), math.radians(35.0)
    v, t = _tilted(theta, phi)
    z = -1.0 if below else 1.0
    w = scenes.plane_workload(proj_eye=(0.0, 0.0, z * 1.0), cam_eye=(0.3, 0.2, z * 1.2), res=32)
    if below:
        w.projector = synth.pinhole((0.0, 0.0, -1.0), (0, 0, 0), 50.0, 32, 32, up=(0, 1, 0))
        w.camera = synth.pinhole((0.3, 0.2, -1.2), (0, 0, 0), 50.0, 32, 32, up=(0, 1, 0))
    w.normal_map = np.tile(v.astype(F32), (8, 8, 1))
    Ep = w.prf_gain * float(np.float32(0.6)) ** 2.2
    rho = 0.5
    n = np.array([0.0, 0.0, z])
    T = np.array([1.0, 0.0, 0.0])
    B = np.cross(n, T)
    vf = v.astype(F32).astype(np.float64)   # the map holds float32 values
    tf = 2 * vf - 1
    ns = (tf[0] * T + tf[1] * B + tf[2] * n) / np.linalg.norm(tf)
    sc = O.Scene(w)
    L = O.render(sc, want=("L",))["L"]
    op = -w.projector.R.T @ w.projector.t
    checked = dark = 0
    for pix in range(32 * 32):
        for s in range(w.spp):
            h = O.first_hit(sc, pix, s)
            if h["prim"] < 0:
                continue
            x = h["x"]
            uv, p = scenes.project(w.projector.K, w.projector.R, w.projector.t, x[None])
            m = min(uv[0][0], 32 - uv[0][0], uv[0][1], 32 - uv[0][1])
            if abs(m) < 1e-6 or m < 0:
                continue
            wp = (op - x) / np.linalg.norm(op - x)
            wo = -h["d"]
            cs, co = ns @ wp, ns @ wo
            if min(abs(cs), abs(co)) < 1e-9:
                continue
            want = rho / math.pi * Ep / p[0, 2] ** 2 * cs / (n @ wp) if (cs > 0 and co > 0) else 0.0
            np.testing.assert_allclose(L[pix, s], want, rtol=1e-11, atol=1e-14)
            checked += 1
            dark += want == 0.0
    assert checked > 2000


def test_flat_normal_map_and_zero_metallic_change_nothing():
    """Maps that encode the unperturbed normal (0.5, 0.5, 1) and metallic 0 give the plain
    BRDF's render and adjoint (to rounding)."""
    w = scenes.c3_ggx(spp=2, seed=9)
    th, tw = w.albedo.shape[:2]
    flat = np.tile(np.array([0.5, 0.5, 1.0], F32), (th, tw, 1))
    base = O.render(O.Scene(w), want=("L",))["L"]
    ext = O.render(O.Scene(w, metallic=np.zeros((th, tw)), normal_map=flat), want=("L",))["L"]
    np.testing.assert_allclose(ext, base, rtol=1e-12, atol=1e-15)
    G = np.random.default_rng(2).normal(size=(64, 64, 3))
    g0 = O.render_vjp(O.Scene(w), G)
    g1 = O.render_vjp(O.Scene(w, metallic=np.zeros((th, tw)), normal_map=flat), G)
    for k in ("Ip", "albedo", "roughness", "specular"):
        np.testing.assert_allclose(g1[k], g0[k], rtol=1e-10, atol=1e-14)


# ---------------------------------------------------------------------------
# adjoint: finite differences on the metallic and normal-map texels
# ---------------------------------------------------------------------------

def ext_workload(spp=3, seed=17, max_depth=3, env=0.3):
    """c3_ggx with a random metallic map and a random normal map (tilts up to ~25 deg)."""
    w = scenes.c3_ggx(spp=spp, seed=seed, max_depth=max_depth)
    rng = np.random.default_rng(77)
    th, tw = w.albedo.shape[:2]
    w.metallic = rng.uniform(0.0, 1.0, (th, tw)).astype(F32)
    t = np.stack([rng.uniform(-0.4, 0.4, (th, tw)), rng.uniform(-0.4, 0.4, (th, tw)), np.ones((th, tw))], -1)
    t /= np.linalg.norm(t, axis=-1, keepdims=True)
    w.normal_map = ((t + 1) / 2).astype(F32)
    w.env = np.array([1.0, 0.8, 0.6]) * env
    w.clip = False
    return w


def test_adjoint_on_metallic_and_normal_map_matches_central_differences():
    """Central differences h = 1e-3 of the frozen-path estimator (directions and pdfs sampled
    with the unperturbed roughness and normal map) on 48 random texels of the metallic and
    normal maps plus 16 of the other maps, GGX, three vertices, environment on."""
    w = ext_workload()
    rng = np.random.default_rng(311)
    G = rng.normal(size=(64, 64, 3))
    base = dict(albedo=w.albedo.astype(np.float64), roughness=w.roughness.astype(np.float64),
                specular=w.specular.astype(np.float64), metallic=w.metallic.astype(np.float64),
                normal_map=w.normal_map.astype(np.float64))
    frozen = dict(rough_sample=base["roughness"], normal_sample=base["normal_map"])
    grad = O.render_vjp(O.Scene(w, **frozen, **base), G)
    th, tw = w.albedo.shape[:2]
    # texels the camera sees through its pixels (the quad spans the whole map)
    picks = []
    for _ in range(24):
        picks.append(("metallic", (int(rng.integers(8, th - 8)), int(rng.integers(8, tw - 8)))))
    for _ in range(24):
        picks.append(("normal_map", (int(rng.integers(8, th - 8)), int(rng.integers(8, tw - 8)), int(rng.integers(0, 3)))))
    for _ in range(16):
        g = ["albedo", "roughness", "specular"][int(rng.integers(0, 3))]
        idx = (int(rng.integers(8, th - 8)), int(rng.integers(8, tw - 8)))
        picks.append((g, idx + ((int(rng.integers(0, 3)),) if g == "albedo" else ())))
    h = 1e-3
    nonzero = 0
    for g, idx in picks:
        def at(delta):
            o = {k: v.copy() for k, v in base.items()}
            o[g][idx] += delta
            out = O.render(O.Scene(w, **frozen, **o), want=("Ic",))
            return float((out["Ic"].reshape(G.shape) * G).sum())
        fd = (at(h) - at(-h)) / (2 * h)
        ad = grad[g][idx]
        assert abs(fd - ad) <= 2e-4 * max(abs(ad), abs(fd)) or abs(fd - ad) < 1e-7, (g, idx, fd, ad)
        nonzero += abs(ad) > 1e-6
    assert nonzero >= 50
